"""Type-II WENO reconstruction on the CSWENO subcell stencils (test oracle).

The paper's subcell stencils are meant to carry any WENO reconstruction
(Sections 1 and 5); type-II schemes combine small-stencil polynomials of a
lower degree than the final one, with linear weights that depend on the
point and can be negative.  This module is the oracle of such a
reconstruction for N = 2 on the stencils of the hierarchical one.  The
paper gives no type-II details; the readings:

* the big stencil is T3 (the nine centroid subcells of the three
  neighbours, Fig. 2a), its quadratic least-squares fit Q with the mean of
  Delta0 exact (the q_3 of Section 3.2);
* six small stencils, each with the mean of Delta0 exact and a linear
  least-squares fit L_j: the three pieces of neighbour k (j = 0, 1, 2) and
  the six pieces of neighbours k, k+1 (j = 3, 4, 5, sectors);
* at every point x where R is evaluated, the linear weights gamma_j(x) are
  the solution of minimal distance to the equal weights 1/6 of
  sum_j gamma_j = 1 and sum_j gamma_j L_j[phi](x) = Q[phi](x) = phi(x) for
  the three quadratic scaled monomials phi (so sum_j gamma_j(x) L_j(x) =
  Q(x) for all data);
* negative weights by the splitting of Shi, Hu and Shu (J. Comput. Phys.
  175, 2002): gamma+ = (gamma + 3 |gamma|) / 2, gamma- = gamma+ - gamma,
  sigma+- = sum gamma+-, nonlinear weights of the WENO-Z form
  omega+-_j = (gamma+-_j / sigma+-) (1 + (tau / (EPS2 + beta_j))^2)
  normalised, tau = max_j beta_j - min_j beta_j, and
  R(x) = sigma+ sum_j omega+_j L_j(x) - sigma- sum_j omega-_j L_j(x)
  (away from extrema the beta_j differ at O(h) relative and omega moves
  off gamma at O(h^2); the classical form gamma_j / (EPS2 + beta_j)^2
  moves at O(h): one application measured 2.66, 2.82, 2.93 against 2.46,
  2.57, 2.67 on 16-128 squares);
* beta_j = |Delta0| |grad L_j|^2 (eq. smoothnessIndicator of a linear
  function);
* R is evaluated at the points of the degree-4 rule on Delta0 and
  projected onto psi_1..psi_5 (the mean is copied); Euler: per
  characteristic field in x and in y, averaged, as the hierarchical one.

Pins (tests/test_oracle_weno_type2.py): the consistency of the linear
weights for quadratics at every point (against the quadratic fit
evaluated directly), the splitting identities, linear data reproduced with
the nonlinear weights, quadratic data reproduced with the linear weights,
the design order on smooth data.  Only tests/ and the benchmark's CPU
baseline use the oracle.
"""
from __future__ import annotations

import numpy as np

from . import basis, quadrature
from .csweno import _solve_ls, monomial_average, monomials, neighbour_average, neighbour_frames, pieces
from .dg import DG, PSI0
from .mesh import INFO_BOUNDARY
from .physics import EQ_EULER, euler_left_eigenvectors, euler_right_eigenvectors, ghost_state

EPS2 = 1.0e-10
THETA = 3.0
NAMES = ["S1", "S2", "S3"]
# small stencils: the faces (neighbours) each one takes
SMALL = [(0,), (1,), (2,), (0, 1), (1, 2), (2, 0)]


def linear_weights(Afit, phi_x):
    """gamma [T, J] at one point: the solution of minimal distance to the
    equal weights of sum_j g_j = 1, sum_j g_j L_j[phi_k](x) = phi_k(x).
    Afit [T, J, 3]: the small fits' values at x of the three quadratic
    monomials' data, phi_x [T, 3] their exact values."""
    T, J, _ = Afit.shape
    A = np.concatenate([np.ones((T, 1, J)), Afit.transpose(0, 2, 1)], axis=1)  # [T, 4, J]
    b = np.concatenate([np.ones((T, 1)), phi_x], axis=1)  # [T, 4]
    g0 = np.full((T, J), 1.0 / J)
    r = b - np.einsum("tij,tj->ti", A, g0)
    # minimal-norm correction: A^T (A A^T)^{-1} r
    AAt = np.einsum("tij,tkj->tik", A, A)
    return g0 + np.einsum("tij,ti->tj", A, np.linalg.solve(AAt, r[..., None])[..., 0])


def split(gamma):
    """Shi-Hu-Shu splitting: gamma = sigma+ g+ - sigma- g- with g+- >= 0
    summing to one."""
    gp = 0.5 * (gamma + THETA * np.abs(gamma))
    gm = gp - gamma
    return gp, gm, gp.sum(axis=-1), gm.sum(axis=-1)


def small_stencil_fits(dg: DG, u, E, characteristic=True):
    """What the type-II and the mixed reconstructions share for the troubled
    cells E (N = 2): Delta0's frame (centroid, mean side, area), the piece
    averages of the three neighbours with the boundary ghosts, the fields
    (characteristic in x and in y for Euler), the mean-free scaled monomial
    averages of the pieces, and the six linear least-squares fits L_j (mean
    of Delta0 exact) with their pseudo-inverses."""
    M = dg.mesh
    T, m = len(E), dg.m
    V0 = M.V[E]
    x0 = V0[:, :, 0].mean(axis=1)
    y0 = V0[:, :, 1].mean(axis=1)
    h0 = M.mean_side[E]
    area0 = M.area[E]
    W, fp, nid, shift = neighbour_frames(dg, E)
    pcs, _ = pieces(W, fp, 1)
    avg = {nm: np.stack([neighbour_average(dg, u, E, nid, shift, f, pcs[nm][:, f]) for f in range(3)], axis=1)
           for nm in NAMES}
    for f in range(3):
        isb = (M.info[E, f] & INFO_BOUNDARY) != 0
        if not isb.any():
            continue
        kind = np.where(isb, M.info[E, f] & 3, 0)
        xm = ym = None
        if dg.shock is not None:
            mid = 0.5 * (M.V[E, f] + M.V[E, (f + 1) % 3])
            xm, ym = mid[:, 0], mid[:, 1]
        for nm in NAMES:
            g = ghost_state(dg.eq, avg[nm][:, f], kind, M.nx[E, f], M.ny[E, f], dg.inflow, dg.shock, xm, ym, dg.time)
            avg[nm][:, f] = np.where(isb[:, None], g, avg[nm][:, f])
    ubar0 = u[E, :, 0] * PSI0

    if dg.eq == EQ_EULER and characteristic:
        dirs = [(1.0, 0.0), (0.0, 1.0)]
        Ls = [euler_left_eigenvectors(ubar0, nx, ny, dg.gamma) for nx, ny in dirs]
        Rs = [euler_right_eigenvectors(ubar0, nx, ny, dg.gamma) for nx, ny in dirs]
    else:
        Ls = [np.broadcast_to(np.eye(m), (T, m, m))]
        Rs = [np.broadcast_to(np.eye(m), (T, m, m))]
    ND = len(Ls)
    to_fields = lambda a: np.concatenate([np.einsum("tij,tkj->tki", Ls[d], a) for d in range(ND)], axis=-1)
    favg = {nm: to_fields(avg[nm]) for nm in NAMES}
    fbar0 = to_fields(ubar0[:, None, :])[:, 0, :]

    mavg0 = monomial_average(V0, x0, y0, h0, 2)
    mavg = {nm: monomial_average(pcs[nm], x0, y0, h0, 2) - mavg0[:, None, :] for nm in NAMES}  # [T, 3 faces, 5]

    def fit(faces, ncol):
        return np.concatenate([mavg[nm][:, list(faces)][..., :ncol] for nm in NAMES], axis=1)

    def data(faces):
        return np.concatenate([favg[nm][:, list(faces)] for nm in NAMES], axis=1) - fbar0[:, None, :]

    # small linear fits: pseudo-inverses X_j [T, 2, rows] and coefficients
    # cL_j [T, 2, F] per field
    Xs, cL = [], []
    for faces in SMALL:
        Q, Rr = np.linalg.qr(fit(faces, 2))
        Xs.append(np.linalg.solve(Rr, Q.transpose(0, 2, 1)))
        cL.append(np.einsum("tcr,trf->tcf", Xs[-1], data(faces)))
    return dict(V0=V0, x0=x0, y0=y0, h0=h0, area0=area0, Ls=Ls, Rs=Rs, ND=ND, favg=favg, fbar0=fbar0,
                mavg0=mavg0, mavg=mavg, fit=fit, data=data, Xs=Xs, cL=cL)


def back_to_conserved(mom, Rs, m):
    """Moments [T, ND*m, n] of the fields back to conserved variables,
    averaged over the ND directions."""
    ND = len(Rs)
    out = 0.0
    for d in range(ND):
        out = out + np.einsum("tij,tjn->tin", Rs[d], mom[:, d * m:(d + 1) * m, :]) / ND
    return out


def reconstruct_type2(dg: DG, u, elems, return_info=False, characteristic=True, linear_only=False):
    """New coefficients [T, m, Np] of the troubled cells elems (mode 0
    copied) by the type-II reconstruction (N = 2)."""
    E = np.asarray(elems, dtype=np.int64)
    T, N, m, Np = len(E), dg.N, dg.m, dg.Np
    if N != 2:
        raise ValueError("the type-II reconstruction is defined for N = 2")
    if T == 0:
        return np.zeros((0, m, Np))
    S = small_stencil_fits(dg, u, E, characteristic)
    V0, x0, y0, h0, area0 = S["V0"], S["x0"], S["y0"], S["h0"], S["area0"]
    ND, fbar0, mavg0, Xs, cL = S["ND"], S["fbar0"], S["mavg0"], S["Xs"], S["cL"]
    mono2 = monomials(2)  # x, y, x^2, xy, y^2 (scaled, mean-free below)
    J = len(SMALL)
    # the quadratic monomials' data through the small fits: L_j[phi_k] coefficients [T, 2] per k
    Lphi = []
    for j, faces in enumerate(SMALL):
        bq = S["fit"](faces, 5)[..., 2:]  # [T, r, 3]: piece averages of phi_k minus Delta0's mean
        Lphi.append(np.einsum("tcr,trk->tck", Xs[j], bq))  # [T, 2, 3]
    beta = [area0[:, None] * np.sum(c * c, axis=1) / h0[:, None] ** 2 for c in cL]  # |grad L|^2 in physical units

    # points of the degree-4 rule on Delta0
    r, s, w = quadrature.triangle_rule_for_degree(4)
    Vh = basis.vandermonde(N, r, s)
    lam1, lam2 = 0.5 * (1.0 + r), 0.5 * (1.0 + s)
    xq = V0[:, 0, 0, None] + lam1 * (V0[:, 1, 0, None] - V0[:, 0, 0, None]) + lam2 * (V0[:, 2, 0, None] - V0[:, 0, 0, None])
    yq = V0[:, 0, 1, None] + lam1 * (V0[:, 1, 1, None] - V0[:, 0, 1, None]) + lam2 * (V0[:, 2, 1, None] - V0[:, 0, 1, None])
    xi = (xq - x0[:, None]) / h0[:, None]
    eta = (yq - y0[:, None]) / h0[:, None]
    phi = np.stack([xi ** a * eta ** b for a, b in mono2], axis=-1) - mavg0[:, None, :]  # [T, q, 5]
    nq = len(w)
    F = ND * m
    Rq = np.zeros((T, nq, F))
    gammas = np.zeros((T, nq, J))
    for q in range(nq):
        Afit = np.stack([np.einsum("tc,tck->tk", phi[:, q, :2], Lphi[j]) for j in range(J)], axis=1)  # [T, J, 3]
        g = linear_weights(Afit, phi[:, q, 2:])
        gammas[:, q] = g
        Lx = np.stack([fbar0 + np.einsum("tc,tcf->tf", phi[:, q, :2], cL[j]) for j in range(J)], axis=1)  # [T, J, F]
        if linear_only:
            Rq[:, q] = np.einsum("tj,tjf->tf", g, Lx)
            continue
        gp, gm, sp, sm = split(g)
        B = np.stack(beta, axis=1)  # [T, J, F]
        tau = B.max(axis=1, keepdims=True) - B.min(axis=1, keepdims=True)
        z = 1.0 + (tau / (EPS2 + B)) ** 2
        wp = (gp / sp[:, None])[..., None] * z
        wm = (gm / sm[:, None])[..., None] * z
        wp = wp / wp.sum(axis=1, keepdims=True)
        wm = wm / wm.sum(axis=1, keepdims=True)
        Rq[:, q] = sp[:, None] * np.sum(wp * Lx, axis=1) - sm[:, None] * np.sum(wm * Lx, axis=1)
    mom = np.einsum("q,tqf,qi->tfi", w, Rq, Vh)
    out = back_to_conserved(mom, S["Rs"], m)
    out[:, :, 0] = u[E, :, 0]
    if return_info:
        return out, dict(cL=cL, Lphi=Lphi, beta=beta, gammas=gammas, phi=phi, fbar0=fbar0, favg=S["favg"],
                         mavg=S["mavg"], mavg0=mavg0, x0=x0, y0=y0, h0=h0, area0=area0, Xs=Xs, rule=(r, s, w))
    return out


def limit_type2(dg: DG, u, mask, characteristic=True, linear_only=False):
    """The type-II limiter on the cells where mask is true (simultaneous)."""
    E = np.nonzero(np.asarray(mask))[0]
    out = u.copy()
    if len(E):
        out[E] = reconstruct_type2(dg, u, E, characteristic=characteristic, linear_only=linear_only)
    return out
