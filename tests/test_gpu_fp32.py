"""FP32-bulk mode (precision 1) against the FP64 oracle (GPU).

In this mode the state is stored in float and the residual and RK combine
compute in float; dt, the KXRCF indicator and the limiter compute in double
from the float state. The oracle runs in FP64 on the same float-rounded
inputs, so:

* dt, flags and R see identical inputs and keep the FP64 bars (dt to 1e-14,
  flags bit-exact, R within 1e-12 on the threshold scale);
* the limiter adds one rounding to float of its FP64 result: normwise
  relative 2 u32 (u32 = 2^-24 = 6.0e-8, the float unit roundoff);
* the residual is a sum of about 20 quadrature contributions per
  coefficient, each from a handful of float operations, so its error is
  bounded by a modest multiple of u32 times the size of the contributions,
  not of the residual (on a nearly steady state, such as the isentropic
  vortex, the residual is a small difference of large flux terms). Each
  contribution is bounded by the element's flux scale (|F| + |G|) P / J
  (cell-mean fluxes, perimeter P, Jacobian J); the bar is 64 u32 = 3.8e-6
  of max(|R|, flux scale) per conserved variable.
"""
import math

import numpy as np
import pytest

from oracle import csweno, kxrcf
from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TOL_RES = 64 * U32
TOL_LIM = 2 * U32 + 1e-12
TIE = 1e-9


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _case(eq, N, n, bc, seed, limiter_mode=0):
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(n, seed=seed)
    M = Mesh(v, t, bc, (1.0, 1.0))
    dg = DG(M, N, eq)
    S = binding.Solver(eq, N, limiter_mode=limiter_mode, precision=1)
    S.mesh_upload(v, t, bc, (1.0, 1.0))
    return M, dg, S


def _f32(u):
    return u.astype(np.float32).astype(np.float64)


def _noisy_state(dg, eq, seed):
    rng = np.random.default_rng(seed)
    if eq == 0:
        u = dg.project(lambda x, y: 0.4 + 0.5 * np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y))
        noise = 0.02
    else:
        u = dg.project(inputs.IsentropicVortex(beta=2.0, x0=0.5, y0=0.5, period_x=1.0, period_y=1.0))
        noise = 0.002
    scale = np.abs(u[:, :, :1]).max(axis=0, keepdims=True)
    u[:, :, 1:] += noise * scale * rng.standard_normal(u[:, :, 1:].shape)
    return _f32(u)


def _jump_state(dg, eq, seed):
    if eq == 0:
        u = dg.project(lambda x, y: 0.3 + 0.5 * np.sin(2 * math.pi * (x + y)) + np.where(x + 0.3 * y > 0.55, 0.8, 0.0))
    else:
        u = dg.project(inputs.FourQuadrant(seed=seed, xc=0.47, yc=0.53, rho_range=(0.6, 1.4),
                                           p_range=(0.6, 1.4), vel_range=(-0.5, 0.5)))
    return _f32(u)


def _flux_scale(M, u, eq):
    """[K, m]: (|F| + |G|) P / J at the cell means."""
    ub = u[:, :, 0] / math.sqrt(2.0)
    if eq == 0:
        F = G = 0.5 * ub ** 2
    else:
        rho, mu, mv, E = ub[:, 0], ub[:, 1], ub[:, 2], ub[:, 3]
        p = 0.4 * (E - 0.5 * (mu * mu + mv * mv) / rho)
        F = np.stack([mu, mu * mu / rho + p, mu * mv / rho, (E + p) * mu / rho], axis=1)
        G = np.stack([mv, mu * mv / rho, mv * mv / rho + p, (E + p) * mv / rho], axis=1)
    return (np.abs(F) + np.abs(G)) * (M.L.sum(axis=1) / M.J)[:, None]


def _reserr(gpu, ref, scale):
    out = []
    for c in range(ref.shape[1]):
        den = max(np.abs(ref[:, c]).max(), scale[:, c].max())
        out.append(np.abs(gpu[:, c] - ref[:, c]).max() / den)
    return max(out)


def _relerr(gpu, ref):
    out = []
    for c in range(ref.shape[1]):
        den = np.abs(ref[:, c]).max()
        out.append(np.abs(gpu[:, c] - ref[:, c]).max() / (den if den > 0 else 1.0))
    return max(out)


EQN = [(0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3)]


def test_fp32_state_is_float(torch):
    M, dg, S = _case(1, 2, 6, BC_PERIODIC, seed=3)
    u = S.to_device(_noisy_state(dg, 1, seed=1))
    assert u.dtype == torch.float32
    assert S.dg_residual(u).dtype == torch.float32
    assert S.project_fn(inputs.IsentropicVortex(beta=2.0, x0=0.5, y0=0.5, period_x=1.0, period_y=1.0)).dtype == torch.float32


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_TRANSMISSIVE])
@pytest.mark.parametrize("eq,N", EQN)
def test_fp32_residual(torch, eq, N, bc):
    M, dg, S = _case(eq, N, 12, bc, seed=41 + N)
    for u in (_noisy_state(dg, eq, seed=N), _jump_state(dg, eq, seed=N)):
        r = S.to_host(S.dg_residual(S.to_device(u)))
        assert _reserr(r, dg.residual(u), _flux_scale(M, u, eq)) < TOL_RES


@pytest.mark.parametrize("eq,N", EQN)
def test_fp32_max_dt(torch, eq, N):
    M, dg, S = _case(eq, N, 10, BC_PERIODIC, seed=51)
    u = _noisy_state(dg, eq, seed=3)
    assert math.isclose(S.max_dt(S.to_device(u)).item(), dg.max_dt(u), rel_tol=1e-14)


@pytest.mark.parametrize("eq,N", EQN)
def test_fp32_kxrcf_flags_bit_exact(torch, eq, N):
    M, dg, S = _case(eq, N, 20, BC_TRANSMISSIVE, seed=61)
    u = _jump_state(dg, eq, seed=5)
    flags, R = S.kxrcf(S.to_device(u))
    flags = flags.cpu().numpy().astype(bool)
    R = R.cpu().numpy()
    Ro, fo = kxrcf.indicator(dg, u)
    ties = np.abs(Ro - 1.0) < TIE
    assert ties.sum() == 0
    assert np.array_equal(flags, fo)
    assert fo.sum() > 0 and (~fo).sum() > 0
    assert np.all(np.abs(R - Ro) <= 1e-12 * np.maximum(Ro, 1.0) + 1e-10)


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_TRANSMISSIVE])
@pytest.mark.parametrize("eq,N", EQN)
def test_fp32_limiter(torch, eq, N, bc):
    M, dg, S = _case(eq, N, 12, bc, seed=71 + N)
    for u in (_jump_state(dg, eq, seed=7), _noisy_state(dg, eq, seed=8)):
        out, _ = S.csweno_limit(S.to_device(u), mask=torch.ones(M.K, dtype=torch.uint8))
        got = S.to_host(out)
        exp = csweno.limit(dg, u, np.ones(M.K, bool))
        assert np.array_equal(got[:, :, 0], u[:, :, 0])  # means copied bitwise
        assert _relerr(got, exp) < TOL_LIM
    # KXRCF-selected cells
    u = _jump_state(dg, eq, seed=9)
    out, flags = S.csweno_limit(S.to_device(u))
    fo = kxrcf.indicator(dg, u)[1]
    assert np.array_equal(flags.cpu().numpy().astype(bool), fo)
    got = S.to_host(out)
    assert np.array_equal(got[~fo], u[~fo])
    assert _relerr(got, csweno.limit(dg, u, fo)) < TOL_LIM


@pytest.mark.parametrize("eq", [0, 1])
@pytest.mark.parametrize("N,kw", [(2, {"reconstruction": 1}), (2, {"reconstruction": 2}), (2, {"reconstruction": 3}),
                                  (3, {"p2_top": 5}), (2, {"beta_mode": 1})])
def test_fp32_limiter_other_readings(torch, eq, N, kw):
    """The other reconstructions and readings read the float state and
    compute in FP64 too: every cell limited against the oracle on the
    float-rounded input, one rounding to float apart."""
    from oracle import weno_mixed, weno_type1, weno_type2
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(10, seed=83)
    M = Mesh(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
    dg = DG(M, N, eq)
    S = binding.Solver(eq, N, precision=1, **kw)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
    u = _jump_state(dg, eq, seed=10)
    out, _ = S.csweno_limit(S.to_device(u), mask=torch.ones(M.K, dtype=torch.uint8))
    allm = np.ones(M.K, bool)
    if kw.get("reconstruction") == 1:
        exp = weno_type1.limit_type1(dg, u, allm)
    elif kw.get("reconstruction") == 2:
        exp = weno_type2.limit_type2(dg, u, allm)
    elif kw.get("reconstruction") == 3:
        exp = weno_mixed.limit_mixed(dg, u, allm)
    else:
        exp = csweno.limit(dg, u, allm, top=binding.top_name(N, kw.get("p2_top", 0)),
                           beta_literal=bool(kw.get("beta_mode", 0)))
    got = S.to_host(out)
    assert np.array_equal(got[:, :, 0], u[:, :, 0])
    assert _relerr(got, exp) < TOL_LIM


@pytest.mark.parametrize("eq,N", [(0, 2), (1, 2)])
def test_fp32_step_all_troubled(torch, eq, N):
    """One SSP-RK3 step with every cell limited (no flag decisions): the
    float stage states differ from the FP64 ones by the residual's float
    error times dt, plus one rounding per stage."""
    M, dg, S = _case(eq, N, 12, BC_PERIODIC, seed=131, limiter_mode=1)
    u = _jump_state(dg, eq, seed=17)
    ud = S.to_device(u)
    dt = dg.max_dt(u)
    lim = lambda v: csweno.limit(dg, v, np.ones(M.K, bool))
    ref = dg.ssprk3_step(u, dt, lim)
    S.ssprk3_step(ud)
    assert _relerr(S.to_host(ud), ref) < TOL_RES
    assert S.status() & 0x7 == 0


def test_fp32_batch_and_graph(torch):
    """Batched instances and a captured graph in FP32-bulk mode: equal bit
    for bit to single-instance eager steps."""
    from paper_2106_06280_amd import binding
    meshes, sol, us = [], [], []
    for i, n in enumerate((5, 8, 6)):
        v, t = inputs.jittered_mesh(n, seed=200 + i)
        meshes.append((v, t))
        S = binding.Solver(1, 2, precision=1)
        S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
        sol.append(S)
        us.append(S.project_fn(inputs.FourQuadrant(seed=i, xc=0.45, yc=0.55, rho_range=(0.6, 1.4),
                                                  p_range=(0.6, 1.4), vel_range=(-0.5, 0.5))))
    B = binding.Solver(1, 2, precision=1)
    B.mesh_upload_batch(meshes, [BC_TRANSMISSIVE] * 3, (1.0, 1.0))
    ub = torch.cat(us, dim=2).contiguous()
    off = B.instances()
    g = binding.Graph([B], [ub], nsteps=2)
    for rep in range(2):
        g.launch()
        for S, u in zip(sol, us):
            S.ssprk3_step(u)
            S.ssprk3_step(u)
        torch.cuda.synchronize()
        for i, u in enumerate(us):
            assert torch.equal(ub[:, :, off[i]:off[i + 1]], u), (rep, i)


def test_fp32_rejects_adjoint(torch):
    from paper_2106_06280_amd import binding
    M, dg, S = _case(1, 2, 5, BC_PERIODIC, seed=7)
    u = S.to_device(_noisy_state(dg, 1, seed=2))
    with pytest.raises(binding.CswdgError):
        S.dg_residual_vjp(u, u.clone())
