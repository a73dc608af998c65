"""TVB minmod troubled-cell indicator on triangles: an addition to the
paper, whose first limiting step is the KXRCF indicator (Section 3.1) and
whose limiter does not depend on which indicator marks the cells (Section
3, the first step; the cited comparison of indicators is where KXRCF is
chosen).  Test infrastructure like the rest of oracle/: only tests, the
smoke check and the benchmark's CPU baseline use it.

The method is the limiter for triangles of Cockburn and Shu (J. Comput.
Phys. 141 (1998) 199-224), used as an indicator as in Zhu, Qiu, Shu and
Dumbser (J. Comput. Phys. 227 (2008) 4330-4353):

1. Element Delta0 has centroid b0; its neighbour across face f has centroid
   b_f (a periodic neighbour translated next to Delta0; across a boundary
   face the mirror image of Delta0, whose centroid is b0 reflected in the
   face).  The midpoint m_i of face i is written as
   m_i - b0 = alpha (b_j - b0) + beta (b_k - b0) with alpha, beta >= 0.  The
   pairs (j, k) are tried in the order (i, i+1), (i, i+2), (i+1, i+2)
   (mod 3); the first whose two coefficients are >= 0 is used, and if none
   is, the pair whose smaller coefficient is largest.
2. Per variable: a_i = u_h(m_i) - ubar0 (the whole polynomial at the
   midpoint) and b_i = alpha (ubar_j - ubar0) + beta (ubar_k - ubar0).
   Across a boundary face the neighbour mean is the ghost's: the mirror
   image keeps ubar0, a reflective wall reverses its normal momentum, an
   inflow face takes the inflow state and a moving-shock face the shock's
   state at the face midpoint and the solution time (the states of the
   boundary kinds of the residual and of the limiter's ghost rows).
3. The TVB-modified minmod m(a, nu b) returns a when |a| <= M h^2, else
   minmod(a, nu b) with nu = 1.5; it leaves a unchanged exactly when
   |a| <= M h^2, or a and b have the same sign and |a| <= nu |b|.  The cell
   is troubled when the minmod would change some a_i of some variable.

Readings (the indicator is not in the paper): h is the circumradius (the h
of the KXRCF test); for the Euler equations each conserved variable is
tested and a cell is troubled if any is; |a_i| at or below 1e-12 times the
cell's largest |mean| counts as no deviation (the rounding left by the
projection of constant data would otherwise flag cells at random), so the
threshold is max(M h^2, 1e-12 max_c |ubar0_c|).

Parity pins (tests/test_oracle_tvb.py): the decomposition reproduces every
midpoint with nonnegative coefficients (neighbour centroids and the ghost
reflection computed independently in the test); global linear data flags
no interior cell; one cell's slope scaled by s is troubled exactly when
s > 1.5 or s < 0 (nu and the sign test); the threshold M h^2 at
the circumradius; constant data flags nothing; a step function flags only
cells that the jump crosses; at a reflective wall, an odd normal momentum
is continued exactly by the ghost (no flags), while an outflow face there
flags.
"""
from __future__ import annotations

import numpy as np

from . import quadrature
from .csweno import neighbour_frames
from .dg import DG, PSI0
from .mesh import INFO_BOUNDARY
from .physics import ghost_state

NU = 1.5
NOISE = 1e-12


def _pairs(i):
    return [(i, (i + 1) % 3), (i, (i + 2) % 3), ((i + 1) % 3, (i + 2) % 3)]


def neighbour_centroids(dg: DG, elems=None):
    """b_f [T, 3, 2]: the placed neighbours' centroids (step 1)."""
    E = np.arange(dg.mesh.K) if elems is None else np.asarray(elems)
    W, _, _, _ = neighbour_frames(dg, E)
    return W.mean(axis=2)


def decomposition(dg: DG, elems=None):
    """A [T, 3, 3] with m_i - b0 = sum_f A[:, i, f] (b_f - b0) (step 1)."""
    M = dg.mesh
    E = np.arange(M.K) if elems is None else np.asarray(elems)
    T = len(E)
    V0 = M.V[E]
    b0 = V0.mean(axis=1)
    d_f = neighbour_centroids(dg, E) - b0[:, None, :]
    A = np.zeros((T, 3, 3))
    rows = np.arange(T)
    for i in range(3):
        d = 0.5 * (V0[:, i] + V0[:, (i + 1) % 3]) - b0
        coef = np.zeros((T, 3, 2))
        low = np.full((T, 3), -np.inf)
        for p, (j, k) in enumerate(_pairs(i)):
            bj, bk = d_f[:, j], d_f[:, k]
            det = bj[:, 0] * bk[:, 1] - bj[:, 1] * bk[:, 0]
            ok = det != 0.0
            sd = np.where(ok, det, 1.0)
            alpha = (d[:, 0] * bk[:, 1] - d[:, 1] * bk[:, 0]) / sd
            beta = (bj[:, 0] * d[:, 1] - bj[:, 1] * d[:, 0]) / sd
            coef[:, p, 0] = np.where(ok, alpha, 0.0)
            coef[:, p, 1] = np.where(ok, beta, 0.0)
            low[:, p] = np.where(ok, np.minimum(alpha, beta), -np.inf)
        nonneg = low >= 0.0
        pick = np.where(nonneg.any(axis=1), nonneg.argmax(axis=1), low.argmax(axis=1))
        for p, (j, k) in enumerate(_pairs(i)):
            sel = pick == p
            A[rows[sel], i, j] = coef[sel, p, 0]
            A[rows[sel], i, k] = coef[sel, p, 1]
    return A


def neighbour_means(dg: DG, u, elems=None):
    """ubar_f [T, 3, m]: the neighbours' cell means, the ghost states' across
    boundary faces (step 2)."""
    M = dg.mesh
    E = np.arange(M.K) if elems is None else np.asarray(elems)
    ub0 = u[E, :, 0] * PSI0
    out = np.zeros((len(E), 3, dg.m))
    for f in range(3):
        isb = (M.info[E, f] & INFO_BOUNDARY) != 0
        nb = np.where(isb, E, M.nbr[E, f])
        kind = np.where(isb, M.info[E, f] & 3, 0)
        mid = 0.5 * (M.V[E, f] + M.V[E, (f + 1) % 3])
        ghost = ghost_state(dg.eq, ub0, kind, M.nx[E, f], M.ny[E, f], dg.inflow, dg.shock, mid[:, 0], mid[:, 1],
                            dg.time)
        out[:, f] = np.where(isb[:, None], ghost, u[nb, :, 0] * PSI0)
    return out


def indicator(dg: DG, u, tvb_m=0.0, elems=None, return_ratio=False):
    """Returns (troubled bool [T], margin [T]), and R [T] with
    return_ratio.  margin is the smallest relative distance of a deciding
    comparison from its tie (|a| against the threshold; |a| against nu |b|
    where the signs agree and |a| is above the threshold): decisions with
    margin below rounding can go either way.  R is the largest ratio of a
    deviation above the threshold to the largest deviation the minmod keeps,
    max(threshold, nu |b| where a b > 0), over midpoints and variables (0 if
    none is above the threshold): troubled exactly when R > 1."""
    M = dg.mesh
    E = np.arange(M.K) if elems is None else np.asarray(elems)
    ub0 = u[E, :, 0] * PSI0  # [T, m]
    A = decomposition(dg, E)
    diff = neighbour_means(dg, u, E) - ub0[:, None, :]  # [T, 3, m]
    b = np.einsum("tif,tfc->tic", A, diff)
    a = np.zeros_like(b)
    for i in range(3):
        r, s = quadrature.face_reference_points(i, np.array([0.0]))
        a[:, i, :] = dg.evaluate(u[E], r, s)[:, 0, :] - ub0
    floor = NOISE * np.abs(ub0).max(axis=1)
    thr = np.maximum(tvb_m * M.circumradius[E] ** 2, floor)[:, None, None]
    absa, nub = np.abs(a), NU * np.abs(b)
    unchanged = (absa <= thr) | ((a * b > 0.0) & (absa <= nub))
    troubled = ~unchanged.all(axis=(1, 2))
    tiny = 1e-300
    d1 = np.abs(absa - thr) / np.maximum(np.maximum(absa, thr), tiny)
    live = (absa > thr) & (a * b > 0.0)
    d2 = np.where(live, np.abs(absa - nub) / np.maximum(np.maximum(absa, nub), tiny), np.inf)
    margin = np.minimum(d1, d2).min(axis=(1, 2))
    if not return_ratio:
        return troubled, margin
    above = absa > thr
    keepmax = np.maximum(thr, np.where(a * b > 0.0, nub, 0.0))
    ratio = np.where(above, absa / np.where(above, keepmax, 1.0), 0.0)
    return troubled, margin, ratio.max(axis=(1, 2))
