"""Pins for fluxes, the Lax-Friedrichs flux and the characteristic matrices
(Section 4 eqs. 2dBurgers, 2dEulerEquations; Section 2 LF flux; Section 3.2
local characteristic decomposition)."""
import numpy as np
import pytest

from oracle import physics as ph


def _state(rng, n):
    rho = rng.uniform(0.2, 2.0, n)
    u = rng.uniform(-1, 1, n)
    v = rng.uniform(-1, 1, n)
    p = rng.uniform(0.1, 2.0, n)
    E = p / 0.4 + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], -1), (rho, u, v, p)


def _fd_jacobian(U, nx, ny, h=1e-6):
    J = np.zeros(U.shape + (4,))
    for k in range(4):
        d = np.zeros(4)
        d[k] = h
        fp, gp = ph.flux(ph.EQ_EULER, U + d)
        fm, gm = ph.flux(ph.EQ_EULER, U - d)
        J[..., :, k] = ((fp - fm) * nx + (gp - gm) * ny) / (2 * h)
    return J


@pytest.mark.parametrize("nx,ny", [(1.0, 0.0), (0.0, 1.0), (0.6, 0.8)])
def test_eigenvectors_diagonalise_fd_jacobian(nx, ny):
    rng = np.random.default_rng(1)
    U, (rho, u, v, p) = _state(rng, 20)
    A = _fd_jacobian(U, nx, ny)
    R = ph.euler_right_eigenvectors(U, nx, ny)
    L = ph.euler_left_eigenvectors(U, nx, ny)
    assert np.allclose(L @ R, np.eye(4), atol=1e-12)
    D = L @ A @ R
    c = np.sqrt(1.4 * p / rho)
    un = u * nx + v * ny
    lam = np.stack([un - c, un, un, un + c], -1)
    assert np.allclose(D, lam[..., None] * np.eye(4), atol=1e-6)
    # fixed scaling: acoustic and entropy columns start with 1; shear column
    # carries a unit tangential velocity
    assert np.allclose(R[:, 0, [0, 1, 3]], 1.0)
    assert np.allclose(R[:, 0, 2], 0.0)
    assert np.allclose(R[:, 1, 2] ** 2 + R[:, 2, 2] ** 2, 1.0)


def test_lax_friedrichs_consistency_and_antisymmetry():
    rng = np.random.default_rng(2)
    a, _ = _state(rng, 30)
    b, _ = _state(rng, 30)
    th = rng.uniform(0, 2 * np.pi, 30)
    nx, ny = np.cos(th), np.sin(th)
    f, g = ph.flux(ph.EQ_EULER, a)
    assert np.allclose(ph.lax_friedrichs(ph.EQ_EULER, a, a, nx, ny), f * nx[:, None] + g * ny[:, None])
    Fab = ph.lax_friedrichs(ph.EQ_EULER, a, b, nx, ny)
    Fba = ph.lax_friedrichs(ph.EQ_EULER, b, a, -nx, -ny)
    assert np.array_equal(Fab, -Fba)
    ub = rng.normal(size=(30, 1))
    ua = rng.normal(size=(30, 1))
    Fab = ph.lax_friedrichs(ph.EQ_BURGERS, ua, ub, nx, ny)
    # Burgers: F.n = u^2/2 (nx + ny), lambda = |u (nx + ny)|
    s = nx + ny
    alpha = np.maximum(np.abs(ua[:, 0] * s), np.abs(ub[:, 0] * s))
    exp = 0.5 * (0.5 * ua[:, 0] ** 2 * s + 0.5 * ub[:, 0] ** 2 * s) - 0.5 * alpha * (ub[:, 0] - ua[:, 0])
    assert np.allclose(Fab[:, 0], exp, rtol=1e-15, atol=1e-15)


def test_euler_flux_closed_form():
    U = np.array([[2.0, 2.0 * 0.5, 2.0 * -0.25, 1.0 / 0.4 + 0.5 * 2.0 * (0.25 + 0.0625)]])
    f, g = ph.flux(ph.EQ_EULER, U)
    # rho=2, u=0.5, v=-0.25, p=1: f = (1, 1.5, -0.25, (E+p)u), g = (-0.5, -0.25, 1.125, (E+p)v)
    E = U[0, 3]
    assert np.allclose(f[0], [1.0, 1.5, -0.25, (E + 1.0) * 0.5])
    assert np.allclose(g[0], [-0.5, -0.25, 1.125, (E + 1.0) * -0.25])
