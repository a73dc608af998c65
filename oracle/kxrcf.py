"""KXRCF troubled-cell indicator (Section 3.1, eq. troubledCellIndicator).

R_j = | int_{dI-} (U_j - U_nb) ds | / ( h^{(N+1)/2} |dI-| ||U_j|| ),
troubled when R_j > C_K with C_K = 1 and h the circumradius.

Readings: the inflow part dI- is taken point by point at the edge Gauss
points (v.n < 0 strictly, v from the interior trace: (u, u) for Burgers,
the velocity for Euler); |dI-| is the same quadrature of 1 over those
points; U is u for Burgers and the density for Euler; ||U_j|| is the
literal L2 norm (int U^2 dA)^(1/2) = (J sum_n U_n^2)^(1/2); R = 0 when
|dI-| = 0 or ||U|| = 0; on a transmissive boundary U_nb = U_j.

Parity status: pinned by tests/test_oracle_kxrcf.py (zero on global
polynomials, closed-form value for a piecewise-constant jump).
"""
from __future__ import annotations

import numpy as np

from . import quadrature
from .dg import DG
from .physics import EQ_BURGERS, moving_shock_state


def indicator(dg: DG, u, elems=None, c_k=1.0, norm="l2"):
    """Returns (R [len], troubled bool [len]).  norm = "l2": the literal
    (int U^2 dA)^(1/2); "rms": the same divided by |Delta|^(1/2), a
    mesh-scale-free variant of the paper's "standard L2 norm"."""
    M = dg.mesh
    E = np.arange(M.K) if elems is None else np.asarray(elems)
    ue = u[E]
    PFrev = dg.PF[:, ::-1, :]
    fprime = M.neighbour_face()
    bnd = M.boundary_mask()
    num = np.zeros(len(E))
    length = np.zeros(len(E))
    for f in range(3):
        um = np.einsum("gn,kcn->kgc", dg.PF[f], ue)
        nb = M.nbr[E, f]
        isb = bnd[E, f]
        nb_safe = np.where(isb, E, nb)
        sel = PFrev[np.where(isb, 0, fprime[E, f])]
        up = np.einsum("kgn,kn->kg", sel, u[nb_safe, 0, :])
        Um = um[..., 0]
        # boundary faces: the ghost state's indicator variable (the interior
        # trace on outflow and wall faces, the inflow state's on inflow
        # faces, the moving shock's state at the point and the solution
        # time on moving-shock faces)
        kind = M.info[E, f] & 3
        Ub = np.where((kind == 2)[:, None], dg.inflow[0], Um)
        if dg.shock is not None and np.any(kind == 3):
            xg, yg = M.physical_points(*quadrature.face_reference_points(f, dg.et), elems=E)
            Ub = np.where((kind == 3)[:, None], moving_shock_state(dg.shock, xg, yg, dg.time)[..., 0], Ub)
        Up = np.where(isb[:, None], Ub, up)
        # inflow points, v.n < 0, as the sign of rho (rho v).(L n) with L n =
        # (ey, -ex) for the edge vector (ex, ey) of face f (L > 0 and rho^2 > 0
        # leave the sign of v.n unchanged; no division); Burgers: v = (u, u)
        ed = M.V[E, (f + 1) % 3] - M.V[E, f]
        ex, ey = ed[:, 0][:, None], ed[:, 1][:, None]
        if dg.eq == EQ_BURGERS:
            sn = Um * (ey - ex)
        else:
            sn = (um[..., 1] * ey - um[..., 2] * ex) * um[..., 0]
        inflow = sn < 0.0
        ds = 0.5 * M.L[E, f][:, None] * dg.ew[None, :]
        num += np.sum(np.where(inflow, ds * (Um - Up), 0.0), axis=1)
        length += np.sum(np.where(inflow, ds, 0.0), axis=1)
    if norm == "rms":
        # int U^2 dA / |Delta| = J sum U_n^2 / (2 J)
        nrm = np.sqrt(0.5 * np.sum(ue[:, 0, :] ** 2, axis=1))
    else:
        nrm = np.sqrt(M.J[E] * np.sum(ue[:, 0, :] ** 2, axis=1))
    h = M.circumradius[E]
    denom = h ** ((dg.N + 1) / 2.0) * length * nrm
    ok = (length > 0.0) & (nrm > 0.0)
    R = np.where(ok, np.abs(num) / np.where(ok, denom, 1.0), 0.0)
    return R, R > c_k
