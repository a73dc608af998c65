"""The matrix-core residual schedule (variant 4: the evaluations at the
quadrature points and the projections onto the test functions as FP64
16x16x4 matrix products over tiles of 16 elements per wave) against the FP64
oracle: every RK stage on periodic and transmissive meshes with a ragged
last tile in every block size, meshes smaller than one tile, the boundary
kinds (walls, inflow, outflow, the moving shock), limited steps, and a
sample of the 1M-element benchmark state.  Bar: 1e-12 normwise per
conserved variable, as for the other schedules."""
import numpy as np
import pytest

from oracle import csweno, kxrcf
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs
from test_gpu_boundaries import SIDES, _case, _dmr_case, _dmr_state, _inflow, _relerr, _state, steps_tol

pytestmark = pytest.mark.gpu

TOL = 1e-12
MATRIX = 4


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _solver(eq, n, bc, seed, block=128, **kw):
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(n, seed=seed)
    M = Mesh(v, t, bc, (1.0, 1.0))
    dg = DG(M, 2, eq)
    S = binding.Solver(eq, 2, **kw)
    S.mesh_upload(v, t, bc, (1.0, 1.0))
    S.set_schedule(MATRIX, block, 1)
    return M, dg, S


def _smooth(dg, eq, seed):
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0.5, 1.5, 2)
    if eq == 0:
        return dg.project(lambda x, y: 0.4 + 0.3 * np.sin(2 * np.pi * (a * x + b * y)))
    return dg.project(lambda x, y: np.stack(
        [1.0 + 0.2 * np.sin(2 * np.pi * (a * x + b * y)), 0.3 + 0.1 * np.cos(2 * np.pi * x),
         -0.2 + 0.1 * np.sin(2 * np.pi * y), 2.5 + 0.3 * np.cos(2 * np.pi * (x - y))], axis=-1))


@pytest.mark.parametrize("block", [64, 128, 256])
@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_TRANSMISSIVE])
@pytest.mark.parametrize("eq", [0, 1])
def test_matrix_residual_and_stages(torch, eq, bc, block):
    """Residual and the three RK combines on 242 elements (15 full tiles of
    16 and a tile of 2; blocks of 16, 32 or 64 elements)."""
    M, dg, S = _solver(eq, 11, bc, seed=301 + eq, block=block)
    assert M.K == 242
    u = _smooth(dg, eq, seed=5) if bc == BC_PERIODIC else _state(dg, eq, seed=5)
    ud = S.to_device(u)
    assert _relerr(S.to_host(S.dg_residual(ud)), dg.residual(u)) < TOL
    prev = _smooth(dg, eq, seed=6)
    pd = S.to_device(prev)
    dt = 0.5 * dg.max_dt(prev)
    dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
    for stage, (a, b) in ((1, (0.0, 1.0)), (2, (0.75, 0.25)), (3, (1.0 / 3.0, 2.0 / 3.0))):
        from paper_2106_06280_amd import binding
        S2 = binding.Solver(eq, 2, limiter_mode=binding.LIMIT_NONE)
        S2.mesh_upload(*inputs.jittered_mesh(11, seed=301 + eq), bc, (1.0, 1.0))
        S2.set_schedule(MATRIX, block, 1)
        out = S2.empty_state()
        S2.rk_stage(stage, ud, pd, out, dtd)
        exp = a * u + b * (prev + dt * dg.residual(prev))
        assert _relerr(S2.to_host(out), exp) < TOL, stage


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("eq", [0, 1])
def test_matrix_meshes_smaller_than_a_block(torch, eq, n):
    """2, 8 and 18 elements: one partly filled tile or two."""
    M, dg, S = _solver(eq, n, BC_TRANSMISSIVE, seed=311 + n)
    u = _state(dg, eq, seed=7)
    assert _relerr(S.to_host(S.dg_residual(S.to_device(u))), dg.residual(u)) < TOL


@pytest.mark.parametrize("eq", [0, 1])
def test_matrix_boundary_kinds(torch, eq):
    """Inflow, outflow and wall faces (the residual's exterior traces)."""
    M, dg, S = _case(eq, 2, 12, 203, SIDES, _inflow(eq))
    S.set_schedule(MATRIX, 128, 1)
    u = _state(dg, eq, seed=3)
    assert _relerr(S.to_host(S.dg_residual(S.to_device(u))), dg.residual(u)) < TOL


def test_matrix_moving_shock(torch):
    """Example 5's boundaries with the moving shock at t = 0.03."""
    M, dg, S = _dmr_case(2, 6, seed=31)
    S.set_schedule(MATRIX, 128, 1)
    T = 0.03
    dg.time = T
    S.set_time(T)
    u = _dmr_state(M, dg, T)
    assert _relerr(S.to_host(S.dg_residual(S.to_device(u))), dg.residual(u)) < TOL


def test_matrix_limited_steps(torch):
    """Three SSP-RK3 steps with KXRCF + CSWENO (four-quadrant data) in the
    matrix schedule against the oracle's steps."""
    M, dg, S = _solver(1, 12, BC_TRANSMISSIVE, seed=321)
    u = _state(dg, 1, seed=9)
    ud = S.to_device(u)
    lim = lambda w: csweno.limit(dg, w, kxrcf.indicator(dg, w)[1])
    for _ in range(3):
        u = dg.ssprk3_step(u, dg.max_dt(u), lim)
        S.ssprk3_step(ud)
    assert S.troubled_stats()[0] > 0
    assert _relerr(S.to_host(ud), u) < steps_tol(3)


def test_matrix_full_size_sample(torch):
    """The benchmark's 999,698-element P2 Euler state (four-quadrant cell
    means after 5 steps): the matrix residual on a 4,000-element sample
    against the oracle, and the whole residual against the compact
    schedule's."""
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(707, seed=1000)
    M = Mesh(v, t, BC_TRANSMISSIVE)
    dg = DG(M, 2, 1)
    S = binding.Solver(binding.EQ_EULER, 2)
    S.mesh_upload(v, t, binding.BC_TRANSMISSIVE)
    ud = S.project_fn(inputs.FourQuadrant(seed=1000))
    ud[:, 1:, :] = 0.0
    for _ in range(5):
        S.ssprk3_step(ud)
    r3 = S.dg_residual(ud).clone()
    S.set_schedule(MATRIX, 128, 1)
    r4 = S.dg_residual(ud)
    u = S.to_host(ud)
    rng = np.random.default_rng(1000)
    sample = np.sort(rng.choice(M.K, 4000, replace=False))
    got = S.to_host(r4[:, :, torch.from_numpy(sample).cuda()])
    err = _relerr(got, dg.residual(u, elems=sample))
    dif = (r4 - r3).abs().amax(dim=(1, 2)) / r3.abs().amax(dim=(1, 2))
    print(f"matrix residual at 1M: sample rel. err. {err:.2e}, against the compact schedule {dif.max().item():.2e}",
          flush=True)
    assert err < TOL
    assert dif.max().item() < TOL
