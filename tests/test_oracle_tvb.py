"""Pins for the TVB minmod troubled-cell indicator (an addition to the
paper, which uses KXRCF; Cockburn-Shu's limiter for triangles used as an
indicator)."""
import numpy as np
import pytest

from oracle import tvb
from oracle.dg import DG, PSI0
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, BKIND_OUTFLOW, BKIND_WALL, INFO_BOUNDARY, Mesh
from paper_2106_06280_amd import inputs


def _mesh(kind, n=8, seed=2):
    if kind == "periodic":
        v, t = inputs.jittered_mesh(n, seed=seed)
        return Mesh(v, t, BC_PERIODIC, (1.0, 1.0))
    if kind == "transmissive":
        v, t = inputs.jittered_mesh(n, seed=seed)
        return Mesh(v, t, BC_TRANSMISSIVE)
    v, t = inputs.forward_step_mesh(5, seed=seed)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(inputs.forward_step_kinds(v, t))
    return M


def _centroids_by_hand(M):
    """b_f by plain loops: the neighbour's vertex mean plus its periodic
    shift, or b0 reflected in the face line (b0 - 2 ((b0 - P) . n) n)."""
    sx, sy = M.neighbour_shift()
    out = np.zeros((M.K, 3, 2))
    for e in range(M.K):
        b0 = M.V[e].sum(axis=0) / 3.0
        for f in range(3):
            if M.info[e, f] & INFO_BOUNDARY:
                n = np.array([M.nx[e, f], M.ny[e, f]])
                out[e, f] = b0 - 2.0 * np.dot(b0 - M.V[e, f], n) * n
            else:
                out[e, f] = M.V[M.nbr[e, f]].sum(axis=0) / 3.0 + np.array([sx[e, f], sy[e, f]])
    return out


@pytest.mark.parametrize("kind", ["periodic", "transmissive", "ffstep"])
def test_decomposition_reproduces_midpoints(kind):
    M = _mesh(kind)
    dg = DG(M, 1, 1)
    A = tvb.decomposition(dg)
    bf = _centroids_by_hand(M)
    h = M.L.max()
    for e in range(M.K):
        b0 = M.V[e].sum(axis=0) / 3.0
        for i in range(3):
            m = 0.5 * (M.V[e, i] + M.V[e, (i + 1) % 3])
            assert np.count_nonzero(A[e, i]) <= 2
            assert A[e, i].min() >= 0.0
            rec = sum(A[e, i, f] * (bf[e, f] - b0) for f in range(3))
            assert np.abs(rec - (m - b0)).max() < 1e-13 * h


def _linear(dg, eq):
    if eq == 0:
        return dg.project(lambda x, y: 0.4 + 0.7 * x - 0.5 * y)
    return dg.project(lambda x, y: np.stack([1.0 + 0.3 * x - 0.2 * y, 0.5 - 0.4 * x + 0.1 * y,
                                             -0.2 + 0.2 * x + 0.6 * y, 3.0 + 0.5 * x + 0.3 * y], axis=-1))


def _interior(M):
    return np.nonzero(~M.boundary_mask().any(axis=1))[0]


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_linear_data_flags_no_interior_cell(N, eq):
    M = _mesh("transmissive", n=6)
    dg = DG(M, N, eq)
    u = _linear(dg, eq)
    tr, margin = tvb.indicator(dg, u)
    inner = _interior(M)
    assert not tr[inner].any()
    assert margin[inner].min() > 0.1  # |a| = |b| < 1.5 |b|: far from the tie


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("N", [1, 2])
def test_one_cell_slope_scaled(N, eq):
    """Linear data with one interior cell's non-mean modes scaled by s: its
    midpoint deviations become s a while the neighbour differences stay a,
    so the cell is troubled exactly when s > 1.5 or s < 0."""
    M = _mesh("transmissive", n=6)
    dg = DG(M, N, eq)
    base = _linear(dg, eq)
    e = _interior(M)[7]
    for s, expect in [(0.0, False), (0.5, False), (1.0, False), (1.45, False), (1.55, True), (2.0, True),
                      (-0.3, True)]:
        u = base.copy()
        u[e, :, 1:] *= s
        tr, margin, R = tvb.indicator(dg, u, elems=[e], return_ratio=True)
        assert bool(tr[0]) == expect, s
        assert margin[0] > 0.01
        # the ratio to the largest deviation kept: s / 1.5 for s > 0, the
        # deviation over the rounding floor for s < 0
        if s > 0:
            assert abs(R[0] - s / 1.5) < 1e-10
        elif s < 0:
            assert R[0] > 1e6
        else:
            assert R[0] == 0.0


def test_threshold_is_m_h_squared_at_the_circumradius():
    M = _mesh("transmissive", n=6)
    dg = DG(M, 1, 0)
    u = _linear(dg, 0)
    e = _interior(M)[5]
    u[e, :, 1:] *= 2.0
    # the cell's largest midpoint deviation, by direct evaluation of the
    # linear polynomial at the face midpoints
    amax = 0.0
    for i in range(3):
        mx, my = 0.5 * (M.V[e, i] + M.V[e, (i + 1) % 3])
        val = 0.4 + 0.7 * mx - 0.5 * my
        mean = 0.4 + 0.7 * M.centroid[e, 0] - 0.5 * M.centroid[e, 1]
        amax = max(amax, 2.0 * abs(val - mean))
    h2 = M.circumradius[e] ** 2
    assert tvb.indicator(dg, u, tvb_m=0.99 * amax / h2, elems=[e])[0][0]
    assert not tvb.indicator(dg, u, tvb_m=1.01 * amax / h2, elems=[e])[0][0]


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("N", [1, 2, 3])
def test_constant_data_flags_nothing(N, eq):
    M = _mesh("periodic", n=7)
    dg = DG(M, N, eq)
    if eq == 0:
        u = dg.project(lambda x, y: 0.7 + 0.0 * x)
    else:
        u = dg.project(inputs.UniformFlow(1.3, 0.4, -0.7, 2.0))
    # the projection leaves rounding in the higher modes
    assert np.abs(u[:, :, 1:]).max() > 0.0
    tr, margin = tvb.indicator(dg, u)
    assert not tr.any() and margin.min() > 0.5


@pytest.mark.parametrize("N", [1, 2, 3])
def test_step_function_flags_only_cut_cells(N):
    M = _mesh("periodic", n=12, seed=5)
    dg = DG(M, N, 0)
    nx, ny, c = 0.8, 0.6, 0.55

    def step(x, y):
        return np.where(nx * x + ny * y > c, 1.0, 0.2)

    u = dg.project(step)
    side = (M.V[..., 0] * nx + M.V[..., 1] * ny) > c  # [K, 3] vertex sides
    cut = side.any(axis=1) & ~side.all(axis=1)
    tr, _ = tvb.indicator(dg, u)
    assert tr.sum() > 0.5 * cut.sum()
    assert not np.any(tr & ~cut)


def _wall_mesh():
    """[0, 1]^2 with a reflective wall at x = 0 and outflow elsewhere."""
    v, t = inputs.jittered_mesh(8, seed=9)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    a = v[t]
    b = v[np.roll(t, -1, axis=1)]
    xm = 0.5 * (a[..., 0] + b[..., 0])
    return M, np.where(xm < 1e-12, BKIND_WALL, BKIND_OUTFLOW)


def test_wall_ghost_continues_odd_normal_momentum():
    """rho = 1, rho u = 0.8 x, rho v = 0.3, E = 4: across the wall x = 0 the
    ghost's mean (normal momentum reversed) equals the odd continuation of
    rho u at the ghost's centroid, so wall cells see linear data and are
    not troubled; with the same faces as outflow the ghost keeps rho u's mean
    and the cells whose slope points at the wall are troubled."""
    M, kinds = _wall_mesh()
    dg = DG(M, 1, 1)
    u = dg.project(lambda x, y: np.stack([1.0 + 0 * x, 0.8 * x, 0.3 + 0 * x, 4.0 + 0 * x], axis=-1))
    wall_cells = np.nonzero(np.any((kinds == BKIND_WALL) & M.boundary_mask(), axis=1))[0]
    assert len(wall_cells) >= 8
    M.set_boundary_kinds(kinds)
    tr, margin = tvb.indicator(dg, u, elems=wall_cells)
    assert not tr.any() and margin.min() > 0.1
    M.set_boundary_kinds(np.zeros_like(kinds))
    tr_out, _ = tvb.indicator(dg, u, elems=wall_cells)
    assert tr_out.sum() >= len(wall_cells) // 2


def test_a_moved_mean_flags_only_its_stencil():
    """The indicator of a cell reads only its own polynomial and its
    immediate neighbours' means: moving one interior cell's mean on linear
    data can flag that cell and its neighbours, and no other cell."""
    M = _mesh("transmissive", n=6)
    dg = DG(M, 2, 0)
    u = _linear(dg, 0)
    e = _interior(M)[9]
    u[e, 0, 0] += 0.3 / PSI0
    tr, _ = tvb.indicator(dg, u)
    near = np.concatenate([[e], M.nbr[e]])
    others = np.setdiff1d(_interior(M), near)
    assert tr[near].any() and not tr[others].any()
