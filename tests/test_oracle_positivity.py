"""Pins for the positivity-preserving scaling (an addition to the paper's
method; Zhang-Shu scaling at the residual's evaluation points)."""
import numpy as np
import pytest

from oracle import positivity
from oracle.dg import DG, PSI0
from oracle.mesh import BC_PERIODIC, Mesh
from paper_2106_06280_amd import inputs


def _dg(N, n=4):
    v, t = inputs.jittered_mesh(n, seed=11)
    return DG(Mesh(v, t, BC_PERIODIC, (1.0, 1.0)), N, 1)


def _pressure(U, g=1.4):
    return (g - 1.0) * (U[..., 3] - 0.5 * (U[..., 1] ** 2 + U[..., 2] ** 2) / U[..., 0])


def _noisy(dg, amp, seed):
    """Uniform flow plus random high modes of relative size amp."""
    u = dg.project(inputs.UniformFlow(1.0, 0.8, -0.3, 0.4))
    rng = np.random.default_rng(seed)
    u[:, :, 1:] += amp * np.abs(u[:, :, :1]) * rng.standard_normal(u[:, :, 1:].shape)
    return u


@pytest.mark.parametrize("N", [1, 2, 3])
def test_positive_cells_are_unchanged(N):
    dg = _dg(N)
    u = _noisy(dg, 0.02, seed=N)
    P = positivity.points_matrix(dg)
    U = np.einsum("qn,kcn->kqc", P, u)
    assert U[..., 0].min() > 1e-3 and _pressure(U).min() > 1e-3
    out, a, b = positivity.scale(dg, u)
    assert np.array_equal(out, u) and a == 0 and b == 0


@pytest.mark.parametrize("N", [1, 2, 3])
def test_scaled_cells_are_positive_and_minimally_scaled(N):
    dg = _dg(N)
    u = _noisy(dg, 0.6, seed=10 + N)
    P = positivity.points_matrix(dg)
    out, a, b = positivity.scale(dg, u)
    assert a > 0 and b > 0
    # means bit for bit
    assert np.array_equal(out[:, :, 0], u[:, :, 0])
    U = np.einsum("qn,kcn->kqc", P, out)
    ubar = out[:, :, 0] * PSI0
    pbar = _pressure(ubar)
    eps = np.minimum(1e-13, np.minimum(ubar[:, 0], pbar))
    eps_p = np.maximum(eps, 1e-10 * pbar)
    assert np.all(U[..., 0].min(axis=1) >= eps - 1e-14)
    assert np.all(_pressure(U).min(axis=1) >= eps_p - 1e-13)
    # minimal: a scaled cell touches a floor at some point (density or
    # pressure), so a larger factor would break positivity
    changed = np.any(out != u, axis=(1, 2))
    gap = np.minimum(U[..., 0].min(axis=1) - eps, _pressure(U).min(axis=1) - eps_p)
    assert np.all(np.abs(gap[changed]) < 1e-12)
    # idempotent up to rounding
    out2, _, _ = positivity.scale(dg, out)
    assert np.abs(out2 - out).max() < 1e-9 * np.abs(out).max()


def test_pressure_factor_against_a_scan():
    """theta for one cell with only the pressure below the floor (density
    positive everywhere): the largest factor on a fine grid of [0, 1] that
    keeps every point's pressure >= eps, against the scaled modes' ratio."""
    dg = _dg(2, n=2)
    P = positivity.points_matrix(dg)
    rng = np.random.default_rng(5)
    cases = 0
    for trial in range(20):
        u = _noisy(dg, 0.0, seed=0)[:1].copy()
        u[0, 1:3, 1:] = 0.9 * rng.standard_normal((2, 5))  # momentum only
        U = np.einsum("qn,cn->qc", P, u[0])
        if U[:, 0].min() <= 0 or _pressure(U).min() >= 0:
            continue
        out, a, b = positivity.scale(dg, u)
        assert a == 0 and b == 1
        theta = out[0, 1, 1:] @ u[0, 1, 1:] / (u[0, 1, 1:] @ u[0, 1, 1:])
        assert np.allclose(out[0, :, 1:], theta * u[0, :, 1:], rtol=1e-14, atol=0)
        grid = np.linspace(0.0, 1.0, 100001)
        ubar = u[0, :, 0] * PSI0
        Ut = ubar[None, None, :] + grid[:, None, None] * (U - ubar)[None]
        okg = np.all(_pressure(Ut) >= max(1e-13, 1e-10 * _pressure(ubar)), axis=1)
        best = grid[np.nonzero(~okg)[0][0] - 1]
        assert best <= theta < best + 1e-5 + 1e-12
        cases += 1
    assert cases >= 5


def test_density_factor_closed_form():
    """Density below the floor, pressure fine once the density is scaled:
    after the scaling the smallest point density equals eps, which fixes
    the factor as (rhobar - eps) / (rhobar - min rho)."""
    dg = _dg(1, n=2)
    P = positivity.points_matrix(dg)
    u = dg.project(inputs.UniformFlow(1.0, 0.0, 0.0, 10.0))[:1].copy()
    u[0, 0, 1] = 2.5  # density mode 1 only: a linear density dipping below zero
    rho = P @ u[0, 0]
    assert rho.min() < 0
    out, a, b = positivity.scale(dg, u)
    assert a == 1
    rbar = u[0, 0, 0] * PSI0
    assert np.isclose(out[0, 0, 1] / u[0, 0, 1], (rbar - 1e-13) / (rbar - rho.min()), rtol=1e-14)
    assert abs((P @ out[0, 0]).min() - 1e-13) < 1e-15


def test_inadmissible_mean_left_alone():
    dg = _dg(2, n=2)
    u = _noisy(dg, 0.6, seed=3)
    u[0, 3, 0] = -1.0  # negative energy mean -> negative mean pressure
    out, _, _ = positivity.scale(dg, u)
    assert np.array_equal(out[0], u[0])
