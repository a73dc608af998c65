"""Pins for the KXRCF indicator (Section 3.1, eq. troubledCellIndicator)."""
import math

import numpy as np

from oracle import kxrcf
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs


def test_zero_on_global_polynomials():
    v, t = inputs.jittered_mesh(5, seed=1)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    for N in (1, 2, 3):
        d = DG(M, N, 0)
        if N == 1:
            U = d.project(lambda x, y: 0.7 + 0.3 * x - 0.2 * y)
        else:
            U = d.project(lambda x, y: 0.7 + 0.3 * x - 0.2 * y + 0.1 * x * y)
        R, tr = kxrcf.indicator(d, U)
        assert R.max() < 1e-10 and not tr.any()


def test_piecewise_constant_jump_closed_form():
    """Burgers with cellwise-constant u > 0: v = (u, u), a face is inflow
    when nx + ny < 0, and R = |sum_inflow L_f (u_e - u_nb)| /
    (h^{(N+1)/2} sum_inflow L_f u_e sqrt(area)) computed here by plain loops."""
    v, t = inputs.jittered_mesh(4, seed=3)
    M = Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    for N in (1, 2):
        d = DG(M, N, 0)
        cval = np.where(M.centroid[:, 0] < 0.5, 1.0, 0.25)
        U = np.zeros((M.K, 1, d.Np))
        U[:, 0, 0] = cval * math.sqrt(2.0)
        R, tr = kxrcf.indicator(d, U)
        Rr, _ = kxrcf.indicator(d, U, norm="rms")
        for e in range(M.K):
            num = 0.0
            ln = 0.0
            for f in range(3):
                if M.nx[e, f] + M.ny[e, f] < 0:
                    num += M.L[e, f] * (cval[e] - cval[M.nbr[e, f]])
                    ln += M.L[e, f]
            if ln == 0:
                exp = exp_rms = 0.0
            else:
                exp = abs(num) / (M.circumradius[e] ** ((N + 1) / 2) * ln * cval[e] * math.sqrt(M.area[e]))
                # the RMS of a constant over the cell is the constant itself
                exp_rms = abs(num) / (M.circumradius[e] ** ((N + 1) / 2) * ln * cval[e])
            assert math.isclose(R[e], exp, rel_tol=1e-12, abs_tol=1e-14)
            assert math.isclose(Rr[e], exp_rms, rel_tol=1e-12, abs_tol=1e-14)
        assert tr.sum() > 0


def test_smooth_data_unflagged_and_jump_flagged_for_euler():
    v, t = inputs.jittered_mesh(16, seed=4)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    d = DG(M, 2, 1)
    U = d.project(inputs.FourQuadrant(states=inputs.RIEMANN_CONFIG3))
    R, tr = kxrcf.indicator(d, U)
    # troubled cells sit next to the quadrant lines only
    c = M.centroid
    near = (np.abs(c[:, 0] - 0.5) < 2.5 / 16) | (np.abs(c[:, 1] - 0.5) < 2.5 / 16)
    assert tr.sum() > 0 and np.all(near[tr])


def test_inflow_points_of_euler_by_velocity_and_normal():
    """The inflow test as the sign of rho (rho v).(L n) selects the points
    where the interior velocity has v.n < 0: an Euler state whose traces
    have a uniform velocity (a, b) (density and energy varying) has R equal
    to a plain loop that takes a face's points as inflow when a n_x + b n_y <
    0 (the velocity is exact here, so no point is a rounding tie)."""
    v, t = inputs.jittered_mesh(5, seed=9)
    M = Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    d = DG(M, 1, 1)
    a, b = 0.3, -0.7
    rho = lambda x, y: 1.0 + 0.4 * np.where(x + 0.2 * y > 0.5, 1.0, 0.0) + 0.1 * np.sin(2 * math.pi * y)
    U = d.project(lambda x, y: np.stack([rho(x, y), a * rho(x, y), b * rho(x, y), 2.5 + 0.0 * x], -1))
    R, _ = kxrcf.indicator(d, U)
    ue = U[:, 0, :]
    for e in range(M.K):
        num = ln = 0.0
        for f in range(3):
            if a * M.nx[e, f] + b * M.ny[e, f] >= 0.0:
                continue
            nb = M.nbr[e, f]
            fp = M.neighbour_face()[e, f]
            for g in range(len(d.ew)):
                um = d.PF[f, g] @ ue[e]
                up = d.PF[fp, len(d.ew) - 1 - g] @ ue[nb]
                ds = 0.5 * M.L[e, f] * d.ew[g]
                num += ds * (um - up)
                ln += ds
        nrm = math.sqrt(M.J[e] * np.sum(ue[e] ** 2))
        exp = abs(num) / (M.circumradius[e] ** 1.0 * ln * nrm) if ln > 0 else 0.0
        assert abs(R[e] - exp) <= 1e-12 * max(1.0, exp), (e, R[e], exp)
