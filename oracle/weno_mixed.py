"""Mixed WENO reconstruction on the CSWENO subcell stencils (test oracle).

The paper names mixed reconstructions beside type-I and type-II ones as
reconstructions its subcell stencils can carry (Sections 1, 3.2 and 5),
by citation only.  A mixed reconstruction combines one polynomial of the
final degree on a big stencil with lower-degree polynomials on small
stencils, with constant positive linear weights: the big stencil's
polynomial enters through p_0 = (Q - sum_j gamma_j L_j) / gamma_0, so that
the linear combination gamma_0 p_0 + sum_j gamma_j L_j is Q whatever the
positive weights.  This module is its oracle for N = 2 on the stencils of
the type-II reading.  The readings:

* big stencil T3 (the nine centroid subcells of the three neighbours), its
  quadratic least-squares fit Q with the mean of Delta0 exact;
* the six small stencils of the type-II reading (the three pieces of one
  neighbour, the six pieces of two neighbours), linear least-squares fits
  L_j with the mean of Delta0 exact;
* linear weights gamma_0 = 0.85 and gamma_j = 0.025 (any positive weights
  summing to one are admissible, as for the paper's own reconstruction);
* smoothness indicators by eq. smoothnessIndicator: beta_0 over the
  derivative orders 1 and 2 of p_0, beta_j = |Delta0| |grad L_j|^2;
* nonlinear weights of the classical form omega_j ~ gamma_j / (EPS + beta_j)^2
  normalised, EPS = 1e-6;
* R = omega_0 p_0 + sum_j omega_j L_j, projected onto psi_1..psi_5 (the
  mean is copied); Euler: per characteristic field in x and in y, averaged,
  as the hierarchical reconstruction.

Pins (tests/test_oracle_weno_mixed.py): Q reproduces quadratic data; the
linear weights give back Q for any data; linear data are reproduced with
the nonlinear weights; the weights and R of one cell against scalar
arithmetic written from the definitions above; the small stencils away
from a jump take the weight across it; the design order on smooth data.
Only tests/ and the benchmark's CPU baseline use the oracle.
"""
from __future__ import annotations

import numpy as np

from . import basis, quadrature
from .csweno import _beta_matrix
from .dg import DG
from .weno_type2 import SMALL, back_to_conserved, small_stencil_fits

GAMMA0 = 0.85
GAMMA_SMALL = 0.025
EPS = 1.0e-6


def reconstruct_mixed(dg: DG, u, elems, return_info=False, characteristic=True, linear_only=False):
    """New coefficients [T, m, Np] of the troubled cells elems (mode 0
    copied) by the mixed reconstruction (N = 2)."""
    E = np.asarray(elems, dtype=np.int64)
    T, N, m, Np = len(E), dg.N, dg.m, dg.Np
    if N != 2:
        raise ValueError("the mixed reconstruction is defined for N = 2")
    if T == 0:
        return np.zeros((0, m, Np))
    S = small_stencil_fits(dg, u, E, characteristic)
    V0, x0, y0, h0, area0 = S["V0"], S["x0"], S["y0"], S["h0"], S["area0"]
    fbar0, mavg0, cL = S["fbar0"], S["mavg0"], S["cL"]
    J = len(SMALL)
    # Q on T3: least squares over the nine pieces, mean of Delta0 exact
    A3 = S["fit"]((0, 1, 2), 5)  # [T, 9, 5]
    Qr, Rr = np.linalg.qr(A3)
    X3 = np.linalg.solve(Rr, Qr.transpose(0, 2, 1))  # [T, 5, 9]
    cQ = np.einsum("tcr,trf->tcf", X3, S["data"]((0, 1, 2)))  # [T, 5, F]
    F = cQ.shape[-1]
    pad = [np.concatenate([c, np.zeros((T, 3, F))], axis=1) for c in cL]  # L_j as [T, 5, F]
    c0 = (cQ - GAMMA_SMALL * sum(pad)) / GAMMA0
    B = _beta_matrix(V0, x0, y0, h0, area0, 2)
    beta = [np.einsum("tif,tij,tjf->tf", c0, B, c0)] + \
           [area0[:, None] * np.sum(c * c, axis=1) / h0[:, None] ** 2 for c in cL]
    gam = np.array([GAMMA0] + [GAMMA_SMALL] * J)
    if linear_only:
        om = np.broadcast_to(gam[None, :, None], (T, J + 1, F))
    else:
        om = gam[None, :, None] / (EPS + np.stack(beta, axis=1)) ** 2  # [T, J+1, F]
        om = om / om.sum(axis=1, keepdims=True)
    cR = om[:, 0][:, None, :] * c0 + sum(om[:, j + 1][:, None, :] * pad[j] for j in range(J))
    # R at the points of the degree-4 rule on Delta0, projected onto P2
    r, s, w = quadrature.triangle_rule_for_degree(4)
    Vh = basis.vandermonde(N, r, s)
    lam1, lam2 = 0.5 * (1.0 + r), 0.5 * (1.0 + s)
    xq = V0[:, 0, 0, None] + lam1 * (V0[:, 1, 0, None] - V0[:, 0, 0, None]) + lam2 * (V0[:, 2, 0, None] - V0[:, 0, 0, None])
    yq = V0[:, 0, 1, None] + lam1 * (V0[:, 1, 1, None] - V0[:, 0, 1, None]) + lam2 * (V0[:, 2, 1, None] - V0[:, 0, 1, None])
    xi = (xq - x0[:, None]) / h0[:, None]
    eta = (yq - y0[:, None]) / h0[:, None]
    phi = np.stack([xi ** a * eta ** b for a, b in [(1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]], axis=-1) \
        - mavg0[:, None, :]  # [T, q, 5]
    Rq = fbar0[:, None, :] + np.einsum("tqk,tkf->tqf", phi, cR)
    mom = np.einsum("q,tqf,qi->tfi", w, Rq, Vh)
    out = back_to_conserved(mom, S["Rs"], m)
    out[:, :, 0] = u[E, :, 0]
    if return_info:
        return out, dict(cQ=cQ, cL=cL, c0=c0, beta=beta, omega=om, cR=cR, X3=X3, B=B, fbar0=fbar0,
                         favg=S["favg"], mavg=S["mavg"], mavg0=mavg0, x0=x0, y0=y0, h0=h0, area0=area0,
                         phi=phi, rule=(r, s, w))
    return out


def limit_mixed(dg: DG, u, mask, characteristic=True, linear_only=False):
    """The mixed limiter on the cells where mask is true (simultaneous)."""
    E = np.nonzero(np.asarray(mask))[0]
    out = u.copy()
    if len(E):
        out[E] = reconstruct_mixed(dg, u, E, characteristic=characteristic, linear_only=linear_only)
    return out
