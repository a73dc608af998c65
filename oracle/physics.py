"""Fluxes, wave speeds and characteristic matrices of the two conservation
laws the paper solves.

* 2D Burgers (Section 4, eq. 2dBurgers): f = g = u^2/2.
* 2D Euler (Section 4, eq. 2dEulerEquations): U = (rho, rho u, rho v, E),
  f = u U + (0, p, 0, p u), g = v U + (0, 0, p, p v),
  p = (gamma - 1)(E - rho (u^2 + v^2)/2), gamma = 1.4.
* Lax-Friedrichs numerical flux (Section 2, 'Lax-Friedrichs flux for all
  the test cases'), read as the local (Rusanov) form
  F*.n = (F(u-).n + F(u+).n)/2 - alpha (u+ - u-)/2,
  alpha = max(lambda(u-, n), lambda(u+, n)).
* Characteristic matrices for the limiter's local characteristic
  decomposition (Section 3.2, last paragraph): right eigenvectors of the
  flux Jacobian in direction n, acoustic and entropy columns scaled to a
  first component of 1, the shear column a unit tangential velocity; the
  left matrix is the numerical inverse (the HIP side uses a closed form).

Parity status: pinned by tests/test_oracle_physics.py (Jacobian by finite
differences, L A R diagonal with the textbook eigenvalues, L R = I).
"""
from __future__ import annotations

import numpy as np

EQ_BURGERS = 0
EQ_EULER = 1


def n_vars(eq: int) -> int:
    return 1 if eq == EQ_BURGERS else 4


def flux(eq, U, gamma=1.4):
    """Physical fluxes (f, g) for states U [..., m]."""
    if eq == EQ_BURGERS:
        h = 0.5 * U * U
        return h, h
    rho, mu, mv, E = U[..., 0], U[..., 1], U[..., 2], U[..., 3]
    u = mu / rho
    v = mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    f = np.stack([mu, mu * u + p, mv * u, (E + p) * u], axis=-1)
    g = np.stack([mv, mu * v, mv * v + p, (E + p) * v], axis=-1)
    return f, g


def normal_speed(eq, U, nx, ny, gamma=1.4):
    """Largest |eigenvalue| of the normal flux Jacobian."""
    if eq == EQ_BURGERS:
        return np.abs(U[..., 0] * (nx + ny))
    rho, mu, mv, E = U[..., 0], U[..., 1], U[..., 2], U[..., 3]
    u = mu / rho
    v = mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(gamma * p / rho)
    return np.abs(u * nx + v * ny) + c


def lax_friedrichs(eq, Um, Up, nx, ny, gamma=1.4, alpha=None):
    """Lax-Friedrichs normal flux F*.n for traces Um (inside), Up: local
    (alpha per point from the two traces) unless a global constant alpha is
    given."""
    fm, gm = flux(eq, Um, gamma)
    fp, gp = flux(eq, Up, gamma)
    nxe = nx[..., None]
    nye = ny[..., None]
    Fm = fm * nxe + gm * nye
    Fp = fp * nxe + gp * nye
    if alpha is None:
        alpha = np.maximum(normal_speed(eq, Um, nx, ny, gamma), normal_speed(eq, Up, nx, ny, gamma))
    else:
        alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), nx.shape)
    return 0.5 * (Fm + Fp) - 0.5 * alpha[..., None] * (Up - Um)


def cell_mean_speed(eq, Ubar, gamma=1.4):
    """Wave-speed bound from a cell-mean state: Burgers sqrt(2)|u|,
    Euler |v| + c."""
    if eq == EQ_BURGERS:
        return np.sqrt(2.0) * np.abs(Ubar[..., 0])
    rho, mu, mv, E = Ubar[..., 0], Ubar[..., 1], Ubar[..., 2], Ubar[..., 3]
    u = mu / rho
    v = mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    return np.sqrt(u * u + v * v) + np.sqrt(gamma * p / rho)


def euler_right_eigenvectors(Ubar, nx, ny, gamma=1.4):
    """R [..., 4, 4] (columns = eigenvectors for u_n - c, u_n, u_n (shear),
    u_n + c) of dF.n/dU at the state Ubar."""
    rho, mu, mv, E = Ubar[..., 0], Ubar[..., 1], Ubar[..., 2], Ubar[..., 3]
    u = mu / rho
    v = mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(gamma * p / rho)
    H = (E + p) / rho
    un = u * nx + v * ny
    one = np.ones_like(rho)
    zero = np.zeros_like(rho)
    r1 = np.stack([one, u - c * nx, v - c * ny, H - c * un], axis=-1)
    r2 = np.stack([one, u, v, 0.5 * (u * u + v * v)], axis=-1)
    r3 = np.stack([zero, -ny * one, nx * one, -ny * u + nx * v], axis=-1)
    r4 = np.stack([one, u + c * nx, v + c * ny, H + c * un], axis=-1)
    return np.stack([r1, r2, r3, r4], axis=-1)


def euler_left_eigenvectors(Ubar, nx, ny, gamma=1.4):
    return np.linalg.inv(euler_right_eigenvectors(Ubar, nx, ny, gamma))


def euler_eigenvalues(Ubar, nx, ny, gamma=1.4):
    rho, mu, mv, E = Ubar[..., 0], Ubar[..., 1], Ubar[..., 2], Ubar[..., 3]
    u = mu / rho
    v = mv / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(gamma * p / rho)
    un = u * nx + v * ny
    return np.stack([un - c, un, un, un + c], axis=-1)


def moving_shock_state(shock, x, y, t):
    """The state on either side of a planar shock moving at constant speed
    (the top boundary of Section 4, Example 5): shock = dict(n=(nx, ny),
    d0=d0, w=w, post=[m], pre=[m]); the post-shock state where
    n.x < d0 + w t, the pre-shock state elsewhere.  x, y [...] -> [..., m]."""
    behind = shock["n"][0] * np.asarray(x) + shock["n"][1] * np.asarray(y) < shock["d0"] + shock["w"] * t
    return np.where(behind[..., None], np.asarray(shock["post"], dtype=np.float64),
                    np.asarray(shock["pre"], dtype=np.float64))


def ghost_state(eq, um, kind, nx, ny, inflow, shock=None, x=None, y=None, t=0.0):
    """Exterior trace at boundary points (Section 4, Examples 4-6).
    um [..., m] interior trace, kind [...] (0 outflow: the interior trace;
    1 reflective wall: the interior trace with its normal momentum reversed;
    2 inflow: the prescribed state inflow [m]; 3 moving shock: the state of
    moving_shock_state at the points x, y [...] and time t), nx, ny [...]
    the outward normal."""
    up = np.array(um, dtype=np.float64, copy=True)
    kind = np.broadcast_to(kind, um.shape[:-1])
    if eq == EQ_EULER:
        mn = um[..., 1] * nx + um[..., 2] * ny
        wall = kind == 1
        up[..., 1] = np.where(wall, um[..., 1] - 2.0 * mn * nx, up[..., 1])
        up[..., 2] = np.where(wall, um[..., 2] - 2.0 * mn * ny, up[..., 2])
    inflow = np.asarray(inflow, dtype=np.float64)
    up = np.where((kind == 2)[..., None], np.broadcast_to(inflow, up.shape), up)
    if shock is not None and np.any(kind == 3):
        up = np.where((kind == 3)[..., None], moving_shock_state(shock, x, y, t), up)
    return up
