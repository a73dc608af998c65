"""Pins for the oracle's DG operator and RK3 (Section 2; end of Section 3,
table:tvd; Section 4.1 Tables 1-2 without limiter)."""
import math
import os

import numpy as np
import pytest

import oracle_runs
from oracle import dg as dgmod
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs


def _poly(N):
    # a global polynomial of degree N and its gradient
    c = {1: (0.3, 0.5, -0.2, 0, 0, 0, 0, 0, 0, 0),
         2: (0.3, 0.5, -0.2, 0.1, 0.3, -0.2, 0, 0, 0, 0),
         3: (0.3, 0.5, -0.2, 0.1, 0.3, -0.2, 0.05, -0.1, 0.07, 0.02)}[N]

    def u(x, y):
        return (c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
                + c[6] * x ** 3 + c[7] * x * x * y + c[8] * x * y * y + c[9] * y ** 3)

    def ux(x, y):
        return c[1] + 2 * c[3] * x + c[4] * y + 3 * c[6] * x * x + 2 * c[7] * x * y + c[8] * y * y

    def uy(x, y):
        return c[2] + c[4] * x + 2 * c[5] * y + c[7] * x * x + 2 * c[8] * x * y + 3 * c[9] * y * y

    return u, ux, uy


@pytest.mark.parametrize("lf", [0, 1])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_burgers_residual_exact_on_global_polynomials(N, lf):
    """Transmissive boundaries and continuous polynomial data: every face
    flux equals the physical flux (whatever the Lax-Friedrichs constant,
    local or global, since the traces agree), so L(u) = Pi_N(-div F(u))
    exactly with the volume and edge rules' degrees (3N-1 and 3N)."""
    v, t = inputs.jittered_mesh(4, -1, 1, -1, 1, seed=2)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    d = DG(M, N, 0)
    d.lf_mode = lf
    u, ux, uy = _poly(N)
    U = d.project(u)
    L = d.residual(U)
    expect = d.project(lambda x, y: -u(x, y) * (ux(x, y) + uy(x, y)))
    assert np.abs(L - expect).max() < 1e-12 * max(1.0, np.abs(expect).max())


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_TRANSMISSIVE])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_euler_freestream(bc, N):
    v, t = inputs.jittered_mesh(4, seed=5)
    M = Mesh(v, t, bc, (1.0, 1.0))
    d = DG(M, N, 1)
    U = d.project(lambda x, y: inputs.primitive_to_conservative(1.3 + 0 * x, 0.4, -0.7, 0.9))
    assert np.abs(d.residual(U)).max() < 1e-12


@pytest.mark.parametrize("lf", [0, 1])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_conservation_periodic(N, lf):
    v, t = inputs.jittered_mesh(5, seed=6)
    M = Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    d = DG(M, N, 1)
    d.lf_mode = lf
    rng = np.random.default_rng(N)
    U = d.project(inputs.IsentropicVortex(beta=2.0, x0=0.5, y0=0.5, period_x=1, period_y=1))
    U[:, :, 1:] += 0.01 * rng.standard_normal(U[:, :, 1:].shape)
    L = d.residual(U)
    tot = np.sum(M.J[:, None] * L[:, :, 0], axis=0)
    scale = np.sum(np.abs(M.J[:, None] * L[:, :, 0]), axis=0)
    assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_rk3_table_matches_golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "rk3_table.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for st, l, a, b in rows:
        i, l = int(st), int(l)
        assert math.isclose(dgmod.RK3_ALPHA[i - 1][l], float(a), rel_tol=1e-15)
        assert math.isclose(dgmod.RK3_BETA[i - 1][l], float(b), rel_tol=1e-15)


def test_rk3_stability_polynomial_and_order():
    for z in (-0.3, -1.0, -2.2, 0.5):
        y = dgmod.ssprk3_step(np.array([1.0]), 1.0, lambda u: z * u)
        assert math.isclose(y[0], 1 + z + z * z / 2 + z ** 3 / 6, rel_tol=1e-14)
    # third order on y' = -y^2, y(0) = 1 -> y = 1/(1+t)
    errs = []
    for n in (10, 20):
        y = np.array([1.0])
        for _ in range(n):
            y = dgmod.ssprk3_step(y, 1.0 / n, lambda u: -u * u)
        errs.append(abs(y[0] - 0.5))
    assert 2.8 < math.log2(errs[0] / errs[1]) < 3.2


def test_max_dt_formula():
    v, t = inputs.jittered_mesh(3, seed=1)
    M = Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    d = DG(M, 2, 0)
    U = d.project(lambda x, y: 0.5 + 0 * x)
    dt = d.max_dt(U)
    assert math.isclose(dt, (0.3 / 5) * np.min(2 * M.inradius) / (math.sqrt(2) * 0.5), rel_tol=1e-14)


ORDERS = oracle_runs.load_orders()


@pytest.mark.parametrize("N", [1, 2, 3])
def test_burgers_convergence_without_limiter(N):
    _, o = oracle_runs.convergence("burgers", N, [8, 16], 0.5 / math.pi, False)
    assert abs(o[-1] - ORDERS[(1, N)][0]) < 0.45, o


@pytest.mark.parametrize("N", [1, 2])
def test_entropy_wave_convergence_without_limiter(N):
    _, o = oracle_runs.convergence("entropy", N, [8, 16], 0.2, False)
    assert abs(o[-1] - ORDERS[(2, N)][0]) < 0.45, o


@pytest.mark.parametrize("N", [1, 2])
def test_global_lax_friedrichs_dissipates_more(N):
    """Burgers, cellwise-constant data on a periodic mesh: the rate of the
    discrete energy sum_e J_e u_e L_e is the flux part minus the
    dissipation alpha/2 |jump|^2 summed over faces, so the global constant
    (the largest cell-mean speed, never below a face's local alpha) gives a
    rate at most the local one's, and strictly below where some face's
    local alpha is smaller."""
    v, t = inputs.jittered_mesh(6, seed=8)
    M = Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    rng = np.random.default_rng(3)
    rates = []
    for lf in (0, 1):
        d = DG(M, N, 0)
        d.lf_mode = lf
        U = np.zeros((M.K, 1, d.Np))
        U[:, 0, 0] = rng.uniform(-1.0, 1.0, M.K) if lf == 0 else U0
        if lf == 0:
            U0 = U[:, 0, 0].copy()
        L = d.residual(U)
        rates.append(np.sum(M.J * U[:, 0, 0] * L[:, 0, 0]))
    assert rates[1] < rates[0] - 1e-6 * abs(rates[0])


def test_step_stage_times_integrate_quadratics_exactly():
    """DG.ssprk3_step evaluates the residual of its stages at t, t + dt and
    t + dt/2 (the times of u^n, u^(1), u^(2) in table:tvd): with a residual
    that depends on time only, one step integrates t^2 exactly and
    advances the solution time by dt."""
    v, t = inputs.jittered_mesh(2, seed=1)
    d = DG(Mesh(v, t, BC_PERIODIC, (1.0, 1.0)), 1, 0)
    d.residual = lambda u, elems=None, t=None: np.full_like(u, t * t)
    d.time = 0.3
    dt = 0.2
    u = np.zeros((d.mesh.K, 1, d.Np))
    out = d.ssprk3_step(u, dt)
    exact = ((0.3 + dt) ** 3 - 0.3 ** 3) / 3.0
    assert np.allclose(out, exact, rtol=1e-14, atol=0)
    assert math.isclose(d.time, 0.5, rel_tol=1e-15)
