"""The TVB minmod troubled-cell indicator (params.indicator = 1; an addition
to the paper, which uses KXRCF) through the C ABI against the oracle (GPU).

Bars: flags bit-exact away from ties (cells whose deciding comparison is
within a relative 1e-9 of equality, counted separately and expected 0);
limited results within 1e-12 normwise of the oracle limiting the same
cells; limited steps within 1e-10."""
import math

import numpy as np
import pytest

from oracle import csweno, tvb
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs

TOL = 1e-12


def steps_tol(nsteps):
    """Bar of free-running multi-step comparisons: every stage reproduces the
    oracle's stage from the same input within TOL (tested separately), and
    from the second stage on each side starts from its own rounding of the
    previous one; the step maps are stable (no measured amplification above
    O(1) per stage), so the differences add up to at most the number of
    stages times TOL."""
    return 3 * nsteps * TOL


pytestmark = pytest.mark.gpu

TIE = 1e-9
EQN = [(0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3)]


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _relerr(gpu, ref):
    out = []
    for c in range(ref.shape[1]):
        den = np.abs(ref[:, c]).max()
        out.append(np.abs(gpu[:, c] - ref[:, c]).max() / (den if den > 0 else 1.0))
    return max(out)


def _case(eq, N, n, bc, seed, **opts):
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(n, seed=seed)
    M = Mesh(v, t, bc, (1.0, 1.0))
    dg = DG(M, N, eq)
    S = binding.Solver(eq, N, indicator=binding.INDICATOR_TVB, **opts)
    S.mesh_upload(v, t, bc, (1.0, 1.0))
    return M, dg, S


def _state(dg, eq, seed):
    """A smooth field with a jump (Burgers) or four-quadrant Riemann data
    plus a smooth perturbation (Euler): flags both in smooth extrema and at
    the discontinuities."""
    if eq == 0:
        return dg.project(lambda x, y: 0.3 + 0.5 * np.sin(2 * math.pi * (x + y)) + np.where(x + 0.3 * y > 0.55, 0.8, 0.0))
    fq = inputs.FourQuadrant(seed=seed, xc=0.47, yc=0.53, rho_range=(0.6, 1.4), p_range=(0.6, 1.4),
                             vel_range=(-0.5, 0.5))

    def fn(x, y):
        s = fq(x, y)
        s[..., 0] *= 1.0 + 0.1 * np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
        return s
    return dg.project(fn)


def _compare(S, dg, u, tvb_m=0.0, mixed=True):
    """flags bit-exact and R within 1e-9 of the oracle's"""
    flags, R = S.kxrcf(S.to_device(u))
    fo, margin, Ro = tvb.indicator(dg, u, tvb_m=tvb_m, return_ratio=True)
    ties = margin < TIE
    assert ties.sum() == 0, ties.sum()
    assert np.array_equal(flags.cpu().numpy().astype(bool), fo)
    R = R.cpu().numpy()
    assert np.all(np.abs(R - Ro) <= 1e-9 * np.maximum(Ro, 1.0))
    assert np.array_equal(R > 1.0, fo)
    if mixed:
        assert fo.sum() > 0 and (~fo).sum() > 0
    return fo


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_TRANSMISSIVE])
@pytest.mark.parametrize("eq,N", EQN)
def test_tvb_flags_bit_exact(torch, eq, N, bc, precision):
    M, dg, S = _case(eq, N, 18, bc, seed=401 + N, precision=precision)
    u = _state(dg, eq, seed=7 + N)
    if precision == 1:
        u = u.astype(np.float32).astype(np.float64)
    fo = _compare(S, dg, u)
    assert S.troubled_count() == int(fo.sum())


@pytest.mark.parametrize("eq,N", [(0, 2), (1, 1), (1, 3)])
def test_tvb_constant_m(torch, eq, N):
    """tvb_m > 0: deviations up to M h^2 (h the circumradius) pass; fewer
    cells are flagged than with M = 0."""
    M, dg, S0 = _case(eq, N, 18, BC_TRANSMISSIVE, seed=411)
    _, _, S = _case(eq, N, 18, BC_TRANSMISSIVE, seed=411, tvb_m=50.0)
    u = _state(dg, eq, seed=3)
    fo = _compare(S, dg, u, tvb_m=50.0)
    f0 = _compare(S0, dg, u)
    assert fo.sum() < f0.sum()


@pytest.mark.parametrize("eq,N", EQN)
def test_limiter_with_tvb_flags(torch, eq, N):
    M, dg, S = _case(eq, N, 14, BC_TRANSMISSIVE, seed=421)
    u = _state(dg, eq, seed=11)
    out, flags = S.csweno_limit(S.to_device(u))
    fo = _compare(S, dg, u)
    assert np.array_equal(flags.cpu().numpy().astype(bool), fo)
    got = S.to_host(out)
    assert np.array_equal(got[~fo], u[~fo])
    assert _relerr(got, csweno.limit(dg, u, fo)) < 1e-12


@pytest.mark.parametrize("eq,N", [(0, 1), (1, 1), (1, 2), (1, 3)])
def test_steps_with_tvb_indicator(torch, eq, N):
    M, dg, S = _case(eq, N, 14, BC_TRANSMISSIVE, seed=431)
    u = _state(dg, eq, seed=13)
    ud = S.to_device(u)
    lim = lambda w: csweno.limit(dg, w, tvb.indicator(dg, w)[0])
    for _ in range(3):
        u = dg.ssprk3_step(u, dg.max_dt(u), lim)
        S.ssprk3_step(ud)
    assert _relerr(S.to_host(ud), u) < steps_tol(3), _relerr(S.to_host(ud), u)
    assert S.status() & 0x3 == 0


def _box(N, n, seed, kinds_lrbt, inflow=None):
    """[0, 1]^2 with boundary kinds per side (left, right, bottom, top)."""
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(n, seed=seed)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    kinds = np.zeros((M.K, 3), dtype=np.int64)
    left, right, bottom, top = kinds_lrbt
    for f in range(3):
        mid = 0.5 * (M.V[:, f] + M.V[:, (f + 1) % 3])
        kinds[:, f] = np.where(mid[:, 0] < 1e-12, left, np.where(mid[:, 0] > 1 - 1e-12, right,
                               np.where(mid[:, 1] < 1e-12, bottom, np.where(mid[:, 1] > 1 - 1e-12, top, 0))))
    M.set_boundary_kinds(kinds)
    dg = DG(M, N, 1)
    dg.inflow = np.zeros(4) if inflow is None else np.asarray(inflow, dtype=np.float64)
    S = binding.Solver(1, N, indicator=binding.INDICATOR_TVB)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
    S.set_boundary(kinds.astype(np.uint8), dg.inflow)
    return M, dg, S


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tvb_wall_ghost(torch, N):
    """Walls on the left and bottom, outflow elsewhere; rho, E constant,
    rho u = 0.8 x, rho v = -0.6 y: the wall ghosts (normal momentum
    reversed) continue the data exactly, so the cells touching only walls
    are not troubled (with outflow ghosts every one of them would be)."""
    M, dg, S = _box(N, 12, 481, (1, 0, 1, 0))
    u = dg.project(lambda x, y: np.stack([1.0 + 0 * x, 0.8 * x, -0.6 * y, 4.0 + 0 * x], axis=-1))
    fo = _compare(S, dg, u)
    k = M.boundary_kind()
    wall_only = (k == 1).any(axis=1) & ~(k == 0).any(axis=1)
    assert wall_only.sum() >= 10 and not fo[wall_only].any()


@pytest.mark.parametrize("N", [1, 2])
def test_tvb_inflow_ghost(torch, N):
    """Inflow on the left of data linear in x: with the inflow state
    U0 - 0.3 h G no inflow cell is troubled, with U0 every one is."""
    G = np.array([0.3, 0.4, 0.2, 0.5])
    U0 = np.array([1.0, 0.6, -0.3, 3.0])
    n = 12
    for kap, expect in [(-0.3, False), (0.0, True)]:
        M, dg, S = _box(N, n, 443, (2, 0, 1, 1), inflow=U0 + kap * G / n)
        u = dg.project(lambda x, y: U0 + x[..., None] * G)
        fo = _compare(S, dg, u, mixed=False)
        infl = (M.boundary_kind() == 2).any(axis=1)
        assert np.all(fo[infl] == expect), kap


@pytest.mark.parametrize("N", [1, 2, 3])
def test_tvb_boundary_kinds_forward_step(torch, N):
    """Example 6's tunnel (walls, inflow, outflow) with the synthetic bow
    shock scaled by a linear factor."""
    from paper_2106_06280_amd import binding
    v, t = inputs.forward_step_mesh(10, seed=441)
    kinds = inputs.forward_step_kinds(v, t)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(kinds)
    dg = DG(M, N, 1)
    ic = inputs.UniformFlow(*inputs.FFSTEP_PRIMITIVE)
    dg.inflow = ic.state
    S = binding.Solver(1, N, indicator=binding.INDICATOR_TVB)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (0.0, 0.0))
    S.set_boundary(kinds.astype(np.uint8), ic.state)
    fs = inputs.ForwardStepShock()
    u = dg.project(lambda x, y: fs(x, y) * (1.0 + 0.05 * x)[..., None])
    _compare(S, dg, u)


def test_tvb_moving_shock(torch):
    """Example 5's boundaries at t = 0.03: the moving shock's state at the
    face midpoints as the ghost mean on the top."""
    from oracle.physics import moving_shock_state
    from paper_2106_06280_amd import binding
    D = inputs.DoubleMachReflection
    v, t = inputs.dmr_mesh(6, seed=451)
    kinds = inputs.dmr_kinds(v, t)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    M.set_boundary_kinds(kinds)
    dg = DG(M, 2, 1)
    sh = D.shock()
    dg.shock, dg.inflow, dg.time = sh, np.asarray(sh["post"]), 0.03
    S = binding.Solver(1, 2, indicator=binding.INDICATOR_TVB)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (0.0, 0.0))
    S.set_moving_shock(sh["post"], sh["pre"], sh["n"], sh["d0"], sh["w"])
    S.set_boundary(kinds.astype(np.uint8), sh["post"])
    S.set_time(0.03)
    u = dg.project(lambda x, y: moving_shock_state(sh, x, y, 0.03) * (1.0 + 0.05 * x)[..., None])
    _compare(S, dg, u)


def test_tvb_batch_equals_instances(torch):
    """A batch with the TVB indicator flags what its instances flag alone
    and steps them identically (bit for bit)."""
    from paper_2106_06280_amd import binding
    meshes, sol, us = [], [], []
    for i, n in enumerate((5, 8, 6)):
        v, t = inputs.jittered_mesh(n, seed=460 + i)
        meshes.append((v, t))
        S = binding.Solver(1, 2, indicator=binding.INDICATOR_TVB)
        S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
        sol.append(S)
        us.append(S.project_fn(inputs.FourQuadrant(seed=20 + i, xc=0.45, yc=0.55, rho_range=(0.6, 1.4),
                                                  p_range=(0.6, 1.4), vel_range=(-0.5, 0.5))))
    B = binding.Solver(1, 2, indicator=binding.INDICATOR_TVB)
    B.mesh_upload_batch(meshes, [BC_TRANSMISSIVE] * 3, (1.0, 1.0))
    ub = torch.cat(us, dim=2).contiguous()
    off = B.instances()
    fb = B.kxrcf(ub)[0]
    for i, (S, u) in enumerate(zip(sol, us)):
        assert torch.equal(fb[off[i]:off[i + 1]], S.kxrcf(u)[0]), i
    for _ in range(2):
        B.ssprk3_step(ub)
        for S, u in zip(sol, us):
            S.ssprk3_step(u)
    for i, u in enumerate(us):
        assert torch.equal(ub[:, :, off[i]:off[i + 1]], u), i


def test_tvb_validation(torch):
    from paper_2106_06280_amd import binding
    with pytest.raises(binding.CswdgError):
        binding.Solver(1, 2, indicator=2)
    with pytest.raises(binding.CswdgError):
        binding.Solver(1, 2, indicator=1, tvb_m=-1.0)
    with pytest.raises(binding.CswdgError):
        binding.Solver(1, 2, indicator=1, tvb_m=float("inf"))
    M, dg, S = _case(1, 2, 6, BC_PERIODIC, seed=471)
    u = S.project_fn(inputs.IsentropicVortex(beta=2.0, x0=0.5, y0=0.5, period_x=1.0, period_y=1.0))
    with pytest.raises(binding.CswdgError):
        S.dg_residual_vjp(u, u.clone())


def test_tvb_and_constant_gamma_in_a_graph(torch):
    """Steps with the TVB indicator and the constant linear weights captured
    in a HIP graph: every replay equals the same steps launched eagerly, bit
    for bit (eager work and synchronisations between the replays)."""
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(14, seed=491)
    S = binding.Solver(1, 2, indicator=binding.INDICATOR_TVB, gamma_mode=1, positivity=1)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
    u0 = S.project_fn(inputs.FourQuadrant(seed=31, xc=0.45, yc=0.55, rho_range=(0.6, 1.4),
                                          p_range=(0.6, 1.4), vel_range=(-0.5, 0.5)))
    ug = u0.clone()
    ue = u0.clone()
    g = binding.Graph([S], [ug], nsteps=2)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for _ in range(2):
            S.ssprk3_step(ue)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
    assert S.status() & 0x3 == 0
