"""Seeded synthetic inputs: jittered triangle meshes and initial/exact states.

This module is the only code shared by the GPU path's callers and by the
CPU oracle.  It produces *data* (vertex coordinates, triangle lists and
pointwise initial states of the conservation law); it contains none of the
discontinuous Galerkin or limiter arithmetic.

Stand-ins for the paper's inputs (Section 4): the paper meshes its domains
with an unstructured generator whose meshes are not available, so every
workload here uses a structured n x n grid of squares, each split along its
(i,j)->(i+1,j+1) diagonal, with interior vertices jittered by a seeded
uniform perturbation of +-0.1 h.  Boundary vertices stay on the uniform grid
so that periodic partners match exactly.

Random numbers come from numpy's PCG64 generator seeded explicitly.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_GAS = 1.4  # ratio of specific heats used for every Euler example (Section 4)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def jittered_mesh(n: int, x0: float = 0.0, x1: float = 1.0, y0: float = 0.0,
                  y1: float = 1.0, jitter: float = 0.1, seed: int = 0,
                  ny: int | None = None):
    """Jittered structured triangulation of [x0,x1] x [y0,y1].

    Returns (vxy, tri): vxy float64 [(n+1)*(ny+1), 2], tri int32 [2*n*ny, 3].
    Vertex (i, j) has id j*(n+1)+i.  Square (i, j) gives the two CCW triangles
    [(i,j),(i+1,j),(i+1,j+1)] and [(i,j),(i+1,j+1),(i,j+1)] with element ids
    2*(j*n+i) and 2*(j*n+i)+1.  Interior vertices move by iid U(-jitter*hx,
    jitter*hx) in x and U(-jitter*hy, jitter*hy) in y.
    """
    if ny is None:
        ny = n
    if n < 1 or ny < 1:
        raise ValueError("mesh needs at least one square per side")
    rng = _rng(seed)
    i = np.arange(n + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    xs = x0 + (x1 - x0) * (i / n)
    ys = y0 + (y1 - y0) * (j / ny)
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # [ny+1, n+1]
    d = rng.uniform(-1.0, 1.0, size=(ny + 1, n + 1, 2))
    hx = (x1 - x0) / n
    hy = (y1 - y0) / ny
    interior = np.zeros((ny + 1, n + 1), dtype=bool)
    interior[1:ny, 1:n] = True
    X = np.where(interior, X + jitter * hx * d[..., 0], X)
    Y = np.where(interior, Y + jitter * hy * d[..., 1], Y)
    vxy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)

    jj, ii = np.meshgrid(np.arange(ny), np.arange(n), indexing="ij")
    a = (jj * (n + 1) + ii).ravel()
    b = a + 1
    c = a + (n + 1) + 1
    dd = a + (n + 1)
    tri = np.empty((2 * n * ny, 3), dtype=np.int32)
    tri[0::2, 0], tri[0::2, 1], tri[0::2, 2] = a, b, c
    tri[1::2, 0], tri[1::2, 1], tri[1::2, 2] = a, c, dd
    return vxy, tri


def forward_step_mesh(s: int, jitter: float = 0.1, seed: int = 0):
    """Wind tunnel of length 4 and width 1 with a step of height 0.2 starting
    1 from the inlet (Section 4, Example 6): [0,4] x [0,1] without the block
    (1,4] x [0,0.2).  Jittered structured triangulation with s squares per
    unit length (s a multiple of 5, so the step's sides lie on grid lines);
    3.4 s^2 squares, 6.8 s^2 triangles.  Vertices strictly inside the
    domain move by iid U(-jitter h, jitter h) per coordinate (h = 1/s);
    vertices on the outer walls, the inlet, the outlet and the step keep
    their places.  Returns (vxy, tri) as jittered_mesh does, unused
    vertices removed."""
    if s < 5 or s % 5:
        raise ValueError("forward_step_mesh: s must be a positive multiple of 5")
    n, ny, js = 4 * s, s, s // 5
    v0, tri = jittered_mesh(n, 0.0, 4.0, 0.0, 1.0, jitter=0.0, ny=ny)
    I = np.tile(np.arange(n + 1), ny + 1)
    J = np.repeat(np.arange(ny + 1), n + 1)
    on_step = ((I == s) & (J <= js)) | ((J == js) & (I >= s))
    in_step = (I > s) & (J < js)
    free = (I > 0) & (I < n) & (J > 0) & (J < ny) & ~on_step & ~in_step
    d = _rng(seed).uniform(-1.0, 1.0, size=(len(v0), 2))
    vxy = v0 + (jitter / s) * d * free[:, None]
    c = v0[tri].mean(axis=1)
    tri = tri[~((c[:, 0] > 1.0) & (c[:, 1] < 0.2))]
    used = np.unique(tri)
    remap = np.full(len(v0), -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return vxy[used].copy(), remap[tri].astype(np.int32)


FFSTEP_OUTFLOW, FFSTEP_WALL, FFSTEP_INFLOW = 0, 1, 2  # boundary kinds, as the solver numbers them


def forward_step_kinds(vxy, tri):
    """[K, 3] boundary kind of face f (vertices f and f+1) of each element of
    a forward_step_mesh: inflow on the inlet x = 0, outflow on the outlet
    x = 4, reflective wall on the tunnel walls and the step (Section 4,
    Example 6).  Entries of interior faces are 1 and are not read."""
    a = vxy[tri]
    b = vxy[np.roll(tri, -1, axis=1)]
    xm = 0.5 * (a[..., 0] + b[..., 0])
    return np.where(xm < 1e-12, FFSTEP_INFLOW, np.where(xm > 4.0 - 1e-12, FFSTEP_OUTFLOW, FFSTEP_WALL))


# Mach 3 uniform flow of the forward-step problem: gamma = 1.4, rho = 1.4,
# p = 1 (sound speed 1), u = 3, v = 0.
FFSTEP_PRIMITIVE = (1.4, 3.0, 0.0, 1.0)


class UniformFlow:
    """Constant state given by primitive variables (rho, u, v, p)."""

    def __init__(self, rho, u, v, p):
        self.state = primitive_to_conservative(rho, u, v, p)

    def __call__(self, x, y):
        return np.broadcast_to(self.state, np.shape(x) + (4,)).copy()


class ForwardStepShock:
    """Synthetic shocked state of the forward-step flow (Section 4, Example 6):
    the uniform Mach 3 flow (FFSTEP_PRIMITIVE) ahead of a curved bow shock
    x = x0 - a y^2 standing in front of the step, and behind it the state
    that a normal shock leaves in that flow (Rankine-Hugoniot jump relations:
    rho2/rho1 = (g+1) M^2 / ((g-1) M^2 + 2), p2/p1 = 1 + 2g (M^2 - 1)/(g+1),
    u2 = u1 rho1/rho2).  x0 ~ U(0.7, 0.9) and a ~ U(0.2, 0.5) from the seed."""

    def __init__(self, seed: int = 0, gamma: float = GAMMA_GAS):
        rng = _rng(seed)
        self.x0 = float(rng.uniform(0.7, 0.9))
        self.a = float(rng.uniform(0.2, 0.5))
        rho1, u1, v1, p1 = FFSTEP_PRIMITIVE
        M2 = u1 * u1 / (gamma * p1 / rho1)
        rho2 = rho1 * (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
        p2 = p1 * (1.0 + 2.0 * gamma * (M2 - 1.0) / (gamma + 1.0))
        self.pre = primitive_to_conservative(rho1, u1, v1, p1, gamma)
        self.post = primitive_to_conservative(rho2, u1 * rho1 / rho2, 0.0, p2, gamma)

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        behind = x > self.x0 - self.a * np.asarray(y) ** 2
        return np.where(behind[..., None], self.post, self.pre)


def n_for_target(k_target: int) -> int:
    """Squares per side so that 2 n^2 is closest to the requested triangle count."""
    return int(round(math.sqrt(k_target / 2.0)))


# ----------------------------------------------------------------------------
# Pointwise states.  Scalar problems return an array shaped like x; Euler
# problems return conservative variables stacked on a trailing axis of 4:
# (rho, rho*u, rho*v, E) with E = p/(gamma-1) + rho*(u^2+v^2)/2 (Section 4,
# Euler equations of Example 2).
# ----------------------------------------------------------------------------

def primitive_to_conservative(rho, u, v, p, gamma=GAMMA_GAS):
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(t, dtype=np.float64) for t in (rho, u, v, p)))
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E], axis=-1)


class BurgersSine:
    """u0 = a + b sin(k (x + y)); with u0 = F(x+y) the exact solution follows
    the characteristics of u_t + 2 u u_xi = 0 in xi = x + y until they cross
    (Example 1 uses a = 0.5, b = 1, k = pi/2 on [-2,2]^2)."""

    def __init__(self, a=0.5, b=1.0, k=math.pi / 2):
        self.a, self.b, self.k = a, b, k

    def __call__(self, x, y):
        return self.a + self.b * np.sin(self.k * (np.asarray(x) + np.asarray(y)))

    def breaking_time(self):
        return 1.0 / (2.0 * self.b * self.k)

    def exact(self, x, y, t, iters=60):
        """Solution at time t by fixed-point/Newton on xi0 + 2 t F(xi0) = xi."""
        xi = np.asarray(x, dtype=np.float64) + np.asarray(y, dtype=np.float64)
        z = xi.copy()
        for _ in range(iters):
            F = self.a + self.b * np.sin(self.k * z)
            dF = self.b * self.k * np.cos(self.k * z)
            g = z + 2.0 * t * F - xi
            z = z - g / (1.0 + 2.0 * t * dF)
        return self.a + self.b * np.sin(self.k * z)


class EntropyWave:
    """Example 2: rho = 1 + 0.2 sin(pi (x + y - t)), u = 0.7, v = 0.3, p = 1.

    The paper prints the exact density with x + y - t; the state is advected
    by (0.7, 0.3), for which x + y moves at speed 1, so both agree."""

    def __init__(self, amp=0.2, k=math.pi, u=0.7, v=0.3, p=1.0):
        self.amp, self.k, self.u, self.v, self.p = amp, k, u, v, p

    def exact(self, x, y, t):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        rho = 1.0 + self.amp * np.sin(self.k * (x + y - (self.u + self.v) * t))
        return primitive_to_conservative(rho, self.u + 0 * rho, self.v + 0 * rho, self.p + 0 * rho)

    def __call__(self, x, y):
        return self.exact(x, y, 0.0)


class IsentropicVortex:
    """Example 3: isentropic vortex of strength beta centred at (x0, y0),
    advected with unit x-velocity; p = rho^gamma.  With period_x the
    vortex is wrapped so that the periodic extension is used."""

    def __init__(self, beta=5.0, x0=5.0, y0=0.0, gamma=GAMMA_GAS, period_x=None, period_y=None):
        self.beta, self.x0, self.y0, self.gamma = beta, x0, y0, gamma
        self.px, self.py = period_x, period_y

    def primitive(self, x, y, t):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        g, b = self.gamma, self.beta
        dx = x - self.x0 - t
        dy = y - self.y0
        if self.px:
            dx = dx - self.px * np.round(dx / self.px)
        if self.py:
            dy = dy - self.py * np.round(dy / self.py)
        r2 = dx * dx + dy * dy
        e = np.exp(1.0 - r2)
        T = 1.0 - (g - 1.0) / (16.0 * g * math.pi ** 2) * b * b * e * e
        rho = T ** (1.0 / (g - 1.0))
        u = 1.0 - b * e * dy / (2.0 * math.pi)
        v = b * e * dx / (2.0 * math.pi)
        p = rho ** g
        return rho, u, v, p

    def exact(self, x, y, t):
        return primitive_to_conservative(*self.primitive(x, y, t), gamma=self.gamma)

    def __call__(self, x, y):
        return self.exact(x, y, 0.0)


class FourQuadrant:
    """Piecewise-constant Riemann data with four quadrants split at (xc, yc),
    following the layout of the paper's two-dimensional Riemann problems
    (Example 7).  States are drawn from the seed unless given explicitly as
    a [4, 4] array of primitive (rho, u, v, p) per quadrant, ordered
    (x>=xc,y>=yc), (x<xc,y>=yc), (x<xc,y<yc), otherwise."""

    def __init__(self, seed=None, states=None, xc=0.5, yc=0.5,
                 rho_range=(0.1, 1.5), p_range=(0.03, 1.5), vel_range=(-1.0, 1.0)):
        if states is None:
            rng = _rng(seed)
            st = np.empty((4, 4))
            st[:, 0] = rng.uniform(*rho_range, size=4)
            st[:, 3] = rng.uniform(*p_range, size=4)
            st[:, 1] = rng.uniform(*vel_range, size=4)
            st[:, 2] = rng.uniform(*vel_range, size=4)
            states = st
        self.states = np.asarray(states, dtype=np.float64)
        self.xc, self.yc = xc, yc

    def quadrant(self, x, y):
        x = np.asarray(x)
        y = np.asarray(y)
        right = x >= self.xc
        top = y >= self.yc
        return np.where(top, np.where(right, 0, 1), np.where(right, 3, 2))

    def __call__(self, x, y):
        q = self.quadrant(x, y)
        s = self.states[q]
        return primitive_to_conservative(s[..., 0], s[..., 1], s[..., 2], s[..., 3])


class ShockEntropyWave:
    """Example 4 (Section 4): a shock at x = 0.125 moving right into density
    sine waves on [0,1]^2, with the printed states (rho, u, v, p) =
    (3.857143, 2.629369, 0, 10.333333) for x < 0.125 and
    (1 + 0.2 sin(16 pi x), 0, 0, 1) otherwise; non-reflecting sides at x = 0
    and x = 1, periodic in y.  The post-shock state is that of a Mach 3
    shock running into rho = 1, p = 1, whose speed the mass jump condition
    gives as shock_speed()."""

    X0 = 0.125
    POST = (3.857143, 2.629369, 0.0, 10.333333)

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        pre = primitive_to_conservative(1.0 + 0.2 * np.sin(16.0 * np.pi * x), 0.0 * x, 0.0 * x, 1.0 + 0.0 * x)
        post = primitive_to_conservative(*self.POST)
        return np.where((x < self.X0)[..., None], post, pre)

    @classmethod
    def shock_speed(cls, rho_pre=1.0):
        rho2, u2 = cls.POST[0], cls.POST[1]
        return rho2 * u2 / (rho2 - rho_pre)


class DoubleMachReflection:
    """Example 5 (Section 4): a right-moving Mach 10 shock in [0,4] x [0,1],
    through (1/6, 0) at 60 degrees to the x axis, into gas at rest with
    rho = 1.4, p = 1 (gamma = 1.4, sound speed 1); behind it the
    normal-shock state of that gas, rho = 8, p = 116.5, velocity 8.25 along
    the shock normal (cos 30, -sin 30).  The shock line moves along its
    normal n = (sin 60, -cos 60) at speed 10: post-shock where
    n.x < n.(1/6, 0) + 10 t.  shock() gives these parameters in the form the
    solver's moving-shock boundary takes."""

    X0 = 1.0 / 6.0
    PRE = (1.4, 0.0, 0.0, 1.0)
    POST = (8.0, 8.25 * np.cos(np.pi / 6.0), -8.25 * np.sin(np.pi / 6.0), 116.5)
    N = (np.sin(np.pi / 3.0), -np.cos(np.pi / 3.0))
    SPEED = 10.0

    @classmethod
    def shock(cls):
        return {"n": cls.N, "d0": cls.N[0] * cls.X0, "w": cls.SPEED,
                "post": primitive_to_conservative(*cls.POST), "pre": primitive_to_conservative(*cls.PRE)}

    def __call__(self, x, y):
        sh = self.shock()
        behind = sh["n"][0] * np.asarray(x) + sh["n"][1] * np.asarray(y) < sh["d0"]
        return np.where(behind[..., None], sh["post"], sh["pre"])


def dmr_mesh(s: int, jitter: float = 0.1, seed: int = 0):
    """[0,4] x [0,1] with s squares per unit length (4 s x s squares,
    8 s^2 triangles), interior vertices jittered (Example 5's domain)."""
    return jittered_mesh(4 * s, 0.0, 4.0, 0.0, 1.0, jitter=jitter, seed=seed, ny=s)


DMR_OUTFLOW, DMR_WALL, DMR_INFLOW, DMR_SHOCK = 0, 1, 2, 3  # boundary kinds, as the solver numbers them


def dmr_kinds(vxy, tri):
    """[K, 3] boundary kinds of Example 5 by face midpoint: inflow of the
    post-shock state at x = 0 and on the bottom for x < 1/6, reflective wall
    on the rest of the bottom, outflow at x = 4, the moving shock's states
    on the top.  Interior entries are 0 and are not read."""
    a = vxy[tri]
    b = vxy[np.roll(tri, -1, axis=1)]
    xm = 0.5 * (a[..., 0] + b[..., 0])
    ym = 0.5 * (a[..., 1] + b[..., 1])
    k = np.zeros(tri.shape, dtype=np.int64)
    k = np.where(ym < 1e-12, np.where(xm < DoubleMachReflection.X0, DMR_INFLOW, DMR_WALL), k)
    k = np.where(ym > 1.0 - 1e-12, DMR_SHOCK, k)
    k = np.where(xm < 1e-12, DMR_INFLOW, k)
    k = np.where(xm > 4.0 - 1e-12, DMR_OUTFLOW, k)
    return k


# Printed initial states of the paper's Example 7 (configurations 3 and 12),
# quadrant order as in FourQuadrant: (rho, u, v, p).
RIEMANN_CONFIG3 = np.array([
    [1.5, 0.0, 0.0, 1.5],
    [0.5323, 1.206, 0.0, 0.3],
    [0.138, 1.206, 1.206, 0.029],
    [0.5323, 0.0, 1.206, 0.3],
])
RIEMANN_CONFIG12 = np.array([
    [0.5313, 0.0, 0.0, 0.4],
    [1.0, 0.7276, 0.0, 1.0],
    [0.8, 0.0, 0.0, 1.0],
    [1.0, 0.0, 0.7276, 1.0],
])


class VortexCircles:
    """Periodic isentropic vortex plus seeded circular jumps: inside each of
    n_circles circles (centres uniform in the domain, radii U[r_lo, r_hi],
    periodic distance) density and pressure are multiplied by a factor
    U[f_lo, f_hi]; overlapping circles multiply."""

    def __init__(self, seed, x0=0.0, x1=10.0, y0=-5.0, y1=5.0, n_circles=8,
                 r_range=(1.0, 2.0), f_range=(2.0, 5.0), beta=5.0):
        rng = _rng(seed)
        self.Lx, self.Ly = x1 - x0, y1 - y0
        self.cx = rng.uniform(x0, x1, size=n_circles)
        self.cy = rng.uniform(y0, y1, size=n_circles)
        self.r = rng.uniform(*r_range, size=n_circles)
        self.f = rng.uniform(*f_range, size=n_circles)
        self.vortex = IsentropicVortex(beta=beta, x0=0.5 * (x0 + x1), y0=0.5 * (y0 + y1),
                                       period_x=self.Lx, period_y=self.Ly)

    def __call__(self, x, y):
        rho, u, v, p = self.vortex.primitive(x, y, 0.0)
        fac = np.ones_like(rho)
        for k in range(len(self.r)):
            dx = np.asarray(x) - self.cx[k]
            dy = np.asarray(y) - self.cy[k]
            dx = dx - self.Lx * np.round(dx / self.Lx)
            dy = dy - self.Ly * np.round(dy / self.Ly)
            fac = np.where(dx * dx + dy * dy < self.r[k] ** 2, fac * self.f[k], fac)
        return primitive_to_conservative(rho * fac, u, v, p * fac)


def random_coefficients(shape, seed, scale=1.0):
    """Seeded normal draws (used as raw modal coefficients in parity tests)."""
    return scale * _rng(seed).standard_normal(size=shape)


# ----------------------------------------------------------------------------
# Batches of independent instances (many small problems advanced together).
# ----------------------------------------------------------------------------

class BurgersSmoothJump:
    """u0 = a + b sin(2 pi (kx x + ky y)) + c 1[x . nhat > s] on [0,1]^2."""

    def __init__(self, a, b, kx, ky, c, nx, ny, s):
        self.a, self.b, self.kx, self.ky, self.c = a, b, kx, ky, c
        self.nx, self.ny, self.s = nx, ny, s

    def __call__(self, x, y):
        x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
        jump = (x * self.nx + y * self.ny > self.s).astype(np.float64)
        return self.a + self.b * np.sin(2 * math.pi * (self.kx * x + self.ky * y)) + self.c * jump


class EulerSmoothJump:
    """rho = 1 + 0.2 sin(2 pi (kx x + ky y)) with a half-plane jump added to
    rho and p; constant velocity."""

    def __init__(self, kx, ky, drho, dp, u, v, nx, ny, s, gamma=GAMMA_GAS):
        self.kx, self.ky, self.drho, self.dp, self.u, self.v = kx, ky, drho, dp, u, v
        self.nx, self.ny, self.s, self.gamma = nx, ny, s, gamma

    def __call__(self, x, y):
        x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
        jump = (x * self.nx + y * self.ny > self.s).astype(np.float64)
        rho = 1.0 + 0.2 * np.sin(2 * math.pi * (self.kx * x + self.ky * y)) + self.drho * jump
        p = 1.0 + self.dp * jump
        return primitive_to_conservative(rho, self.u, self.v, p, self.gamma)


def batch_instances(n_inst=256, seed=1004, k_lo=2000, k_hi=60000, n_burgers=None):
    """Seeded descriptions of independent instances on [0,1]^2: the first
    n_burgers (default half) are Burgers (periodic), the rest Euler
    (transmissive).  Triangle counts are drawn log-uniformly in [k_lo, k_hi].
    Each entry: dict(eq, bc, n, mesh_seed, ic)."""
    rng = _rng(seed)
    if n_burgers is None:
        n_burgers = n_inst // 2
    out = []
    for i in range(n_inst):
        k = math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))
        n = max(2, n_for_target(k))
        mesh_seed = int(rng.integers(1 << 31))
        th = rng.uniform(0.0, 2 * math.pi)
        nx, ny = math.cos(th), math.sin(th)
        # the half-plane boundary passes through a point of the unit square
        px, py = rng.uniform(0.25, 0.75, size=2)
        s = nx * px + ny * py
        kx, ky = (int(t) for t in rng.integers(1, 3, size=2))
        if i < n_burgers:
            ic = BurgersSmoothJump(a=rng.uniform(0.2, 0.8), b=rng.uniform(0.1, 0.5), kx=kx, ky=ky,
                                   c=rng.uniform(-0.5, 0.5), nx=nx, ny=ny, s=s)
            out.append(dict(eq=0, bc=0, n=n, mesh_seed=mesh_seed, ic=ic))
        else:
            u, v = rng.uniform(-0.5, 0.5, size=2)
            ic = EulerSmoothJump(kx=kx, ky=ky, drho=rng.uniform(0.2, 1.0), dp=rng.uniform(0.2, 1.0),
                                 u=u, v=v, nx=nx, ny=ny, s=s)
            out.append(dict(eq=1, bc=1, n=n, mesh_seed=mesh_seed, ic=ic))
    return out
