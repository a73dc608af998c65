"""Type-I WENO reconstruction on the CSWENO subcell stencils (test oracle).

The paper states that its compact subcell stencils work with any WENO
reconstruction, naming type-I reconstructions (Section 1, Section 3.2 and
Section 5: every small stencil reconstructs a polynomial of the same degree
as the final one, and the final order is not higher than theirs) beside the
Zhu-Shu hierarchical one it uses.  This module is the oracle of such a
reconstruction built on the same stencils; the weighting follows the
classical WENO form omega_k ~ lambda_k / (eps + beta_k)^r.  Readings (the
paper gives no type-I details):

* small stencils over the centroid subcells Delta_f1, Delta_f2, Delta_f3 of
  the three neighbours (the pieces of T3, Fig. 3): the central stencil takes
  all nine pieces, sector k (k = 0, 1, 2) the six pieces of the neighbours
  across faces k and k+1 (mod 3);
* on each stencil the polynomial of degree N (N = 1, 2) with the mean of
  Delta0 exact and the piece averages matched in the least-squares sense,
  in the scaled monomials of the hierarchical reconstruction;
* beta_k = sum over derivative orders 1..N of |Delta0|^{|a|-1} int (D^a q_k)^2
  (eq. smoothnessIndicator applied to q_k);
* omega_k = lambda_k / (EPS1 + beta_k)^R1 normalised, lambda = LAMBDA_C for
  the central stencil and 1 for the sectors; R = sum_k omega_k q_k;
* the moments 1..Np-1 are the L2 projection of R, the mean is copied; Euler:
  per characteristic field in x and in y, averaged (as the hierarchical
  reconstruction).

Every small stencil reproduces polynomials of degree N, so the
reconstruction reproduces them for any weights: that, the weights in closed
form and the design order on smooth data pin this module
(tests/test_oracle_weno_type1.py).  Only tests/ and the benchmark's CPU
baseline use the oracle.
"""
from __future__ import annotations

import numpy as np

from . import basis, quadrature
from .csweno import (_beta_matrix, _solve_ls, monomial_average, monomials, neighbour_average, neighbour_frames,
                     pieces)
from .dg import DG, PSI0
from .mesh import INFO_BOUNDARY
from .physics import EQ_EULER, euler_left_eigenvectors, euler_right_eigenvectors, ghost_state

# weights omega_k ~ lambda_k / (EPS1 + beta_k)^R1: a large linear weight on
# the central stencil (smooth data take its reconstruction), one on each
# sector, a fourth power of the smoothness indicators and a small epsilon
LAMBDA_C = 1.0e5
EPS1 = 1.0e-14
R1 = 4

SECTORS = [(0, 1), (1, 2), (2, 0)]
NAMES = ["S1", "S2", "S3"]


def reconstruct_type1(dg: DG, u, elems, return_info=False, characteristic=True):
    """New coefficients [T, m, Np] of the troubled cells elems (mode 0
    copied from u) by the type-I WENO reconstruction of degree N on the
    centroid subcells of the three neighbours (N = 1, 2)."""
    M = dg.mesh
    E = np.asarray(elems, dtype=np.int64)
    T, N, m, Np = len(E), dg.N, dg.m, dg.Np
    if N not in (1, 2):
        raise ValueError("the type-I reconstruction is defined for N = 1, 2")
    if T == 0:
        return np.zeros((0, m, Np))
    V0 = M.V[E]
    x0 = V0[:, :, 0].mean(axis=1)
    y0 = V0[:, :, 1].mean(axis=1)
    h0 = M.mean_side[E]
    area0 = M.area[E]
    W, fp, nid, shift = neighbour_frames(dg, E)
    pcs, _ = pieces(W, fp, 1)  # the three centroid subcells of every neighbour

    # averages of every component over the pieces, boundary ghosts as in the
    # hierarchical reconstruction (mirror image; wall, inflow, moving shock)
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
    favg = {nm: to_fields(avg[nm]) for nm in NAMES}  # [T, 3 faces, F]
    fbar0 = to_fields(ubar0[:, None, :])[:, 0, :]  # [T, F]
    F = ND * m

    mono = monomials(N)
    nm_ = len(mono)
    mavg0 = monomial_average(V0, x0, y0, h0, N)  # [T, n]
    mavg = {nm: monomial_average(pcs[nm], x0, y0, h0, N) - mavg0[:, None, :] for nm in NAMES}  # [T, 3, n]

    def fit(faces):
        A = np.concatenate([mavg[nm][:, faces] for nm in NAMES], axis=1)  # rows: piece-major, then face
        b = np.concatenate([favg[nm][:, faces] for nm in NAMES], axis=1) - fbar0[:, None, :]
        return _solve_ls(A, b)  # [T, n, F]

    stencils = [list(range(3))] + [list(s) for s in SECTORS]
    lam = np.array([LAMBDA_C] + [1.0] * len(SECTORS))
    cs = [fit(s) for s in stencils]
    B = _beta_matrix(V0, x0, y0, h0, area0, N)
    betas = [np.einsum("tif,tij,tjf->tf", c, B, c) for c in cs]
    wt = [lam[k] / (EPS1 + betas[k]) ** R1 for k in range(len(cs))]
    ws = sum(wt)
    omega = [w / ws for w in wt]
    Rc = sum(omega[k][:, None, :] * cs[k] for k in range(len(cs)))  # [T, n, F]

    # L2 projection of R = fbar0 + sum_j Rc_j (phi_j - avg phi_j) onto psi_i
    r, s, w = quadrature.triangle_rule_for_degree(2 * N)
    Vh = basis.vandermonde(N, r, s)
    lam1, lam2 = 0.5 * (1.0 + r), 0.5 * (1.0 + s)
    xq = V0[:, 0, 0, None] + lam1 * (V0[:, 1, 0, None] - V0[:, 0, 0, None]) + lam2 * (V0[:, 2, 0, None] - V0[:, 0, 0, None])
    yq = V0[:, 0, 1, None] + lam1 * (V0[:, 1, 1, None] - V0[:, 0, 1, None]) + lam2 * (V0[:, 2, 1, None] - V0[:, 0, 1, None])
    xi = (xq - x0[:, None]) / h0[:, None]
    eta = (yq - y0[:, None]) / h0[:, None]
    phi = np.stack([xi ** a * eta ** b for a, b in mono], axis=-1) - mavg0[:, None, :]
    Rq = fbar0[:, None, :] + np.einsum("tqn,tnf->tqf", phi, Rc)
    mom = np.einsum("q,tqf,qi->tfi", w, Rq, Vh)
    out = np.zeros((T, m, Np))
    for d in range(ND):
        out += np.einsum("tij,tjn->tin", Rs[d], mom[:, d * m:(d + 1) * m, :]) / ND
    out[:, :, 0] = u[E, :, 0]
    if return_info:
        return out, dict(cs=cs, betas=betas, omega=omega, lam=lam, Rc=Rc, favg=favg, fbar0=fbar0, mavg=mavg,
                         mavg0=mavg0, x0=x0, y0=y0, h0=h0, area0=area0, n_mono=nm_)
    return out


def limit_type1(dg: DG, u, mask, characteristic=True):
    """The type-I limiter on the cells where mask is true (simultaneous)."""
    E = np.nonzero(np.asarray(mask))[0]
    out = u.copy()
    if len(E):
        out[E] = reconstruct_type1(dg, u, E, characteristic=characteristic)
    return out
