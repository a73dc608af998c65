"""Pins for the boundary kinds of Section 4's Examples 4-6 (outflow,
reflective wall, inflow): conservation and steady states that the ghost
states must preserve, a closed form of KXRCF at an inflow face, and the
wall ghost of the limiter on wall-symmetric data."""
import math

import numpy as np
import pytest

from oracle import csweno, kxrcf
from oracle.dg import DG
from oracle.mesh import BC_TRANSMISSIVE, BKIND_INFLOW, BKIND_OUTFLOW, BKIND_WALL, Mesh
from oracle.physics import ghost_state
from paper_2106_06280_amd import inputs


def _box(n=6, seed=3):
    v, t = inputs.jittered_mesh(n, seed=seed)
    return Mesh(v, t, BC_TRANSMISSIVE)


def _kinds_by_side(M, left, right, bottom, top):
    """Boundary kind of each face from the side of the unit square it lies on."""
    kinds = np.zeros((M.K, 3), dtype=np.int64)
    for f in range(3):
        mid = 0.5 * (M.V[:, f] + M.V[:, (f + 1) % 3])
        kinds[:, f] = np.where(mid[:, 0] < 1e-12, left,
                               np.where(mid[:, 0] > 1 - 1e-12, right,
                                        np.where(mid[:, 1] < 1e-12, bottom, np.where(mid[:, 1] > 1 - 1e-12, top, 0))))
    return kinds


def test_ghost_state_definitions():
    um = np.array([[1.2, 0.3, -0.4, 2.5]])
    nx, ny = np.array([0.6]), np.array([0.8])
    w = ghost_state(1, um, np.array([1]), nx, ny, np.zeros(4))
    # reflection: same density, energy and tangential momentum; normal reversed
    assert w[0, 0] == 1.2 and w[0, 3] == 2.5
    assert math.isclose(w[0, 1] * nx[0] + w[0, 2] * ny[0], -(0.3 * 0.6 - 0.4 * 0.8), rel_tol=1e-15)
    assert math.isclose(-w[0, 1] * ny[0] + w[0, 2] * nx[0], -0.3 * 0.8 - 0.4 * 0.6, rel_tol=1e-15)
    assert np.array_equal(ghost_state(1, um, np.array([0]), nx, ny, np.zeros(4)), um)
    assert np.array_equal(ghost_state(1, um, np.array([2]), nx, ny, np.arange(4.0)), np.arange(4.0)[None])


@pytest.mark.parametrize("N", [1, 2])
def test_uniform_flow_along_walls_is_steady(N):
    """Walls at y = 0, 1, inflow of the same state at x = 0, outflow at x = 1."""
    M = _box()
    M.set_boundary_kinds(_kinds_by_side(M, BKIND_INFLOW, BKIND_OUTFLOW, BKIND_WALL, BKIND_WALL))
    d = DG(M, N, 1)
    state = inputs.primitive_to_conservative(1.2, 0.8, 0.0, 1.0)
    d.inflow = state
    u = d.project(lambda x, y: np.broadcast_to(state, np.shape(x) + (4,)))
    assert np.abs(d.residual(u)).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_closed_box_conserves_mass_and_energy(N):
    """Walls all round: no mass or energy crosses a reflective wall, whatever
    the state (the reflected ghost has the opposite normal velocity and the
    same density and energy)."""
    M = _box()
    M.set_boundary_kinds(_kinds_by_side(M, BKIND_WALL, BKIND_WALL, BKIND_WALL, BKIND_WALL))
    d = DG(M, N, 1)
    u = d.project(inputs.FourQuadrant(seed=5, xc=0.45, yc=0.55, rho_range=(0.6, 1.4), p_range=(0.6, 1.4),
                                      vel_range=(-0.5, 0.5)))
    R = d.residual(u)
    tot = np.sum(M.J[:, None] * R[:, :, 0], axis=0)  # d/dt of the integrals (times sqrt 2)
    scale = np.sum(M.J[:, None] * np.abs(R[:, :, 0]), axis=0)
    assert abs(tot[0]) < 1e-13 * scale[0]
    assert abs(tot[3]) < 1e-13 * scale[3]
    # the momentum is not conserved: the walls push
    assert abs(tot[1]) > 1e-6 * scale[1]


def test_kxrcf_at_inflow_face_closed_form():
    """Burgers, cellwise-constant u > 0 on a transmissive box with an inflow
    state u_in on the left side: plain loops with the inflow state across
    the left faces and the interior value across the other boundary faces."""
    v, t = inputs.jittered_mesh(4, seed=3)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(_kinds_by_side(M, BKIND_INFLOW, BKIND_OUTFLOW, BKIND_OUTFLOW, BKIND_OUTFLOW))
    for N in (1, 2):
        d = DG(M, N, 0)
        d.inflow = np.array([0.2])
        cval = np.where(M.centroid[:, 0] < 0.5, 1.0, 0.4)
        U = np.zeros((M.K, 1, d.Np))
        U[:, 0, 0] = cval * math.sqrt(2.0)
        R, tr = kxrcf.indicator(d, U)
        kind = M.boundary_kind()
        for e in range(M.K):
            num = ln = 0.0
            for f in range(3):
                if M.nx[e, f] + M.ny[e, f] < 0:
                    if kind[e, f] < 0:
                        other = cval[M.nbr[e, f]]
                    elif kind[e, f] == BKIND_INFLOW:
                        other = 0.2
                    else:
                        other = cval[e]
                    num += M.L[e, f] * (cval[e] - other)
                    ln += M.L[e, f]
            exp = 0.0 if ln == 0 else abs(num) / (M.circumradius[e] ** ((N + 1) / 2) * ln * cval[e] * math.sqrt(M.area[e]))
            assert math.isclose(R[e], exp, rel_tol=1e-12, abs_tol=1e-14)
        left = np.any(kind == BKIND_INFLOW, axis=1)
        assert tr[left].any()


@pytest.mark.parametrize("N", [1, 2])
def test_wall_ghost_reproduces_wall_symmetric_linear_data(N):
    """Linear data with rho, m_x, E even and m_y odd about the wall y = 0:
    the reflected mirror ghost is then the data's own linear extension, so
    the cells touching the wall reproduce it (characteristic limiting)."""
    M = _box(7)
    M.set_boundary_kinds(_kinds_by_side(M, BKIND_OUTFLOW, BKIND_OUTFLOW, BKIND_WALL, BKIND_OUTFLOW))
    d = DG(M, N, 1)
    f = lambda x, y: np.stack([1.0 + 0.2 * x, 0.3 + 0.1 * x, 0.25 * y, 2.5 + 0.1 * x], -1)
    U = d.project(f)
    kind = M.boundary_kind()
    wall = np.nonzero(np.any(kind == BKIND_WALL, axis=1) & ~np.any((kind == BKIND_OUTFLOW), axis=1))[0]
    assert len(wall) > 0
    out = csweno.reconstruct(d, U, wall)
    assert np.abs(out - U[wall]).max() < 1e-11
    # with the wall treated as an outflow (plain mirror) the odd momentum is
    # not reproduced
    M.set_boundary_kinds(np.zeros((M.K, 3), dtype=np.int64))
    out0 = csweno.reconstruct(d, U, wall)
    assert np.abs(out0 - U[wall]).max() > 1e-6


def test_inflow_ghost_is_the_inflow_state():
    """Constant interior data equal to the inflow state is left unchanged by
    the limiter next to an inflow face; a different inflow state changes it."""
    M = _box(6)
    M.set_boundary_kinds(_kinds_by_side(M, BKIND_INFLOW, BKIND_OUTFLOW, BKIND_OUTFLOW, BKIND_OUTFLOW))
    d = DG(M, 2, 1)
    state = inputs.primitive_to_conservative(1.1, 0.5, 0.1, 0.9)
    d.inflow = state
    U = d.project(lambda x, y: np.broadcast_to(state, np.shape(x) + (4,)) + np.stack(
        [0.05 * x * y, 0.0 * x, 0.0 * x, 0.0 * x], -1))
    kind = M.boundary_kind()
    cells = np.nonzero(np.any(kind == BKIND_INFLOW, axis=1))[0]
    out = csweno.reconstruct(d, U, cells)
    d.inflow = state * 1.3
    out2 = csweno.reconstruct(d, U, cells)
    assert np.abs(out2 - out).max() > 1e-6
    assert np.array_equal(out[:, :, 0], U[cells][:, :, 0])


@pytest.mark.parametrize("N", [1, 2])
def test_forward_step_uniform_mach3_closed_form(N):
    """Uniform Mach 3 flow in the forward-step tunnel (Section 4, Example 6)
    with the inflow state equal to it: the residual vanishes except in the
    cells on the step's vertical face, where the wall meets the flow head-on.
    There the reflected ghost carries the opposite normal momentum, so the
    LF flux has no mass or energy part and x-momentum flux
    rho u^2 + p + alpha rho u with alpha = |u| + c.  The rates of the domain
    integrals are then inlet minus outlet (length 1 and 0.8) minus that wall
    flux over the step height 0.2:
    mass 0.2 rho u, x-momentum 0.2 (rho u^2 + p) - 0.2 (rho u^2 + p + 4 rho u),
    energy 0.2 (E + p) u."""
    v, t = inputs.forward_step_mesh(10, seed=3)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(inputs.forward_step_kinds(v, t))
    d = DG(M, N, 1)
    rho, u0, _, p = inputs.FFSTEP_PRIMITIVE
    ic = inputs.UniformFlow(*inputs.FFSTEP_PRIMITIVE)
    d.inflow = ic.state.copy()
    U = d.project(ic)
    R = d.residual(U)
    # integrals: the mean mode times the cell's Jacobian times sqrt 2
    assert math.isclose(math.sqrt(2.0) * np.sum(M.J * U[:, 0, 0]), rho * 3.4, rel_tol=1e-13)
    rate = math.sqrt(2.0) * np.sum(M.J[:, None] * R[:, :, 0], axis=0)
    E = p / 0.4 + 0.5 * rho * u0 * u0
    exp = [0.2 * rho * u0, 0.2 * (rho * u0 * u0 + p) - 0.2 * (rho * u0 * u0 + p + 4.0 * rho * u0), 0.0,
           0.2 * (E + p) * u0]
    assert np.allclose(rate, exp, rtol=1e-12, atol=1e-12)
    kind = M.boundary_kind()
    a, b = M.V, np.roll(M.V, -1, axis=1)
    xm, ym = 0.5 * (a[..., 0] + b[..., 0]), 0.5 * (a[..., 1] + b[..., 1])
    head_on = np.any((kind == BKIND_WALL) & (np.abs(xm - 1.0) < 1e-12) & (ym < 0.2), axis=1)
    assert head_on.sum() == 2
    assert np.abs(R[~head_on]).max() < 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("N", [1, 2])
def test_moving_shock_boundary_matches_the_moving_shock(N):
    """Moving-shock faces all round (Example 5's top boundary kind) and the
    exact planar shock of Example 5 at time t as data: with the solution
    time t the ghost agrees with the data on every boundary face, so every
    cell whose faces all lie on one side of the shock line has a zero
    residual; with the time left at 0 the boundary cells the shock has
    passed since then see the old (pre-shock) ghost and do not."""
    from oracle.physics import moving_shock_state
    D = inputs.DoubleMachReflection
    v, t = inputs.dmr_mesh(5, seed=2)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(np.full((M.K, 3), 3))
    d = DG(M, N, 1)
    d.shock = D.shock()
    T = 0.05
    U = d.project(lambda x, y: moving_shock_state(d.shock, x, y, T))
    n = np.array(d.shock["n"])
    side = M.V @ n - (d.shock["d0"] + d.shock["w"] * T)  # [K, 3] vertex sides
    clear = np.all(side < -1e-12, axis=1) | np.all(side > 1e-12, axis=1)
    nb_clear = np.array([all(clear[j] for j in M.nbr[e] if j >= 0) for e in range(M.K)])
    away = clear & nb_clear
    U[~clear, :, 1:] = 0.0  # cells the line cuts: cell means (no Gibbs undershoot)
    d.time = T
    R = d.residual(U)
    assert away.sum() > 0.5 * M.K
    assert np.abs(R[away]).max() < 1e-10 * np.abs(R).max()
    d.time = 0.0
    R0 = d.residual(U)
    mid = 0.5 * (M.V + np.roll(M.V, -1, axis=1)) @ n  # [K, 3] face midpoints along n
    swept = M.boundary_mask() & (mid > d.shock["d0"] + 1e-12) & (mid < d.shock["d0"] + d.shock["w"] * T - 1e-12)
    passed = swept.any(axis=1) & np.all(side < -1e-12, axis=1)
    assert passed.sum() > 0
    assert np.all(np.abs(R0[passed]).max(axis=(1, 2)) > 1e-6)
