"""Positivity-preserving scaling of Euler polynomials: an addition, not part
of the paper (which has no positivity limiter).  Test infrastructure like
the rest of oracle/: only tests, the smoke check and the benchmark's CPU
baseline use it.

The method is Zhang and Shu's (J. Comput. Phys. 229 (2010) 8918-8934) as
extended to triangles by Zhang, Xia and Shu (J. Sci. Comput. 50 (2012)
29-62): with the cell mean Ubar admissible, the modes above the mean are
scaled towards it until density and pressure reach their floors at
every point where the residual evaluates the solution (its volume points
and the Gauss points of the three edges):

1. eps = min(1e-13, rhobar, pbar); a cell whose mean has rhobar <= 0,
   pbar <= 0 or a non-finite value is left as it is;
2. theta1 = min(1, (rhobar - eps) / (rhobar - min_q rho_q)) scales the
   density's modes 1..Np-1;
3. with that density, each point q whose pressure is below the pressure
   floor eps_p = max(eps, 1e-10 pbar) gets the t_q in [0, 1] at which the
   pressure of (1 - t) Ubar + t U_q equals eps_p;
   the pressure is concave in U where rho > 0, so there is exactly one such
   t, found here by bisection to machine precision; theta2 = min_q t_q (1
   if no point is below eps_p);
4. theta2 scales the modes 1..Np-1 of every variable.

The cell mean (mode 0) is untouched, bit for bit.  The pressure floor is
relative to the mean pressure, not Zhang and Shu's absolute 1e-13: near
vacuum points (small rho_q) the pressure changes fast along the segment,
and the rounding of the root then leaves the pressure up to about 1e-12
away from the floor, below zero with a floor of 1e-13.

Parity pins (tests/test_oracle_positivity.py): cells that are already
positive come back unchanged; after scaling every point is at or above
the floors (up to rounding) and touches one of them and the means are unchanged; a one-cell case with linear
density has theta1 in closed form; the pressure step against a brute-force
scan of t.
"""
from __future__ import annotations

import numpy as np

from .dg import DG, PSI0

EPS_FLOOR = 1e-13


def points_matrix(dg: DG):
    """psi_n at the residual's evaluation points: the volume points, then the
    Gauss points of faces 0, 1, 2: [n_points, Np]."""
    return np.concatenate([dg.V] + [dg.PF[f] for f in range(3)], axis=0)


def _pressure(U, gamma):
    return (gamma - 1.0) * (U[..., 3] - 0.5 * (U[..., 1] ** 2 + U[..., 2] ** 2) / U[..., 0])


def scale(dg: DG, u, iters=64):
    """Return (u', n_density, n_pressure): u with the scaling applied to
    every cell, and the numbers of cells whose density (theta1 < 1) and
    whose modes (theta2 < 1) were scaled."""
    if dg.m != 4:
        raise ValueError("positivity scaling is defined for the Euler equations")
    g = dg.gamma
    P = points_matrix(dg)
    out = np.array(u, dtype=np.float64, copy=True)
    ubar = out[:, :, 0] * PSI0  # [K, 4]
    pbar = _pressure(ubar, g)
    ok = np.isfinite(ubar).all(axis=1) & np.isfinite(pbar) & (ubar[:, 0] > 0) & (pbar > 0)
    eps = np.minimum(EPS_FLOOR, np.minimum(ubar[:, 0], pbar))

    # 1-2: density
    rho_q = np.einsum("qn,kn->kq", P, out[:, 0, :])
    rmin = rho_q.min(axis=1)
    low = ok & (rmin < eps)
    theta1 = np.ones(len(out))
    theta1[low] = (ubar[low, 0] - eps[low]) / (ubar[low, 0] - rmin[low])
    out[:, 0, 1:] *= theta1[:, None]

    # 3-4: pressure
    U = np.einsum("qn,kcn->kqc", P, out)  # [K, q, 4]
    p_q = _pressure(U, g)
    eps_p = np.maximum(eps, 1e-10 * pbar)
    below = ok[:, None] & (p_q < eps_p[:, None])
    theta2 = np.ones(len(out))
    rows = np.nonzero(below.any(axis=1))[0]
    if len(rows):
        Ub = ubar[rows][:, None, :]
        dU = U[rows] - Ub
        e = eps_p[rows][:, None]
        lo = np.zeros(dU.shape[:2])
        hi = np.ones(dU.shape[:2])
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            good = _pressure(Ub + mid[..., None] * dU, g) >= e
            lo = np.where(good, mid, lo)
            hi = np.where(good, hi, mid)
        t = np.where(below[rows], lo, 1.0)
        theta2[rows] = t.min(axis=1)
    out[:, :, 1:] *= theta2[:, None, None]
    return out, int((theta1 < 1).sum()), int((theta2 < 1).sum())
