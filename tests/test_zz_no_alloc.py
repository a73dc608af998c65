"""The allocation-free limiter entry point (cswdg_csweno_limit_noalloc)
against cswdg_csweno_limit on the same inputs: two calls in a row on
different solvers, the second with a smaller mesh, with KXRCF flags and with
a given mask; and the rejection of a mesh whose scratch exceeds the static
array."""
import math

import numpy as np
import pytest

from oracle.dg import DG
from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, Mesh
from paper_2106_06280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _solver(eq, N, n, bc, seed, **kw):
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(n, seed=seed)
    S = binding.Solver(eq, N, **kw)
    S.mesh_upload(v, t, bc, (1.0, 1.0))
    dg = DG(Mesh(v, t, bc, (1.0, 1.0)), N, eq)
    if eq == 0:
        u = dg.project(lambda x, y: 0.3 + 0.5 * np.sin(2 * math.pi * (x + y)) + np.where(x + 0.3 * y > 0.55, 0.8, 0.0))
    else:
        u = dg.project(inputs.FourQuadrant(seed=seed, xc=0.47, yc=0.53, rho_range=(0.6, 1.4), p_range=(0.6, 1.4),
                                           vel_range=(-0.5, 0.5)))
    return S, S.to_device(u)


def _both(torch, S, u, mask=None):
    ref, fref = S.csweno_limit(u, mask=mask)
    out = torch.empty_like(u)
    flags = torch.empty(S.K, dtype=torch.uint8, device="cuda")
    out, flags = S.csweno_limit_noalloc(u, out, flags, mask=mask)
    return ref, fref, out, flags


@pytest.mark.parametrize("N,kw", [(2, {"reconstruction": 1}), (2, {"reconstruction": 2}), (2, {"reconstruction": 3}),
                                  (3, {"p2_top": 5}), (2, {"beta_mode": 1})])
def test_noalloc_limiter_other_readings(torch, N, kw):
    """The entry point runs the solver's own reconstruction: type-I,
    type-II, mixed, the sextic top, the printed smoothness indicators."""
    for n, seed in ((12, 43), (7, 44)):
        S, u = _solver(1, N, n, BC_TRANSMISSIVE, seed, **kw)
        ref, fref, out, flags = _both(torch, S, u)
        assert int(fref.sum()) > 0
        assert torch.equal(flags, fref) and torch.equal(out, ref)


@pytest.mark.parametrize("eq,N,bc", [(1, 2, BC_TRANSMISSIVE), (0, 1, BC_PERIODIC), (1, 3, BC_PERIODIC)])
def test_noalloc_limiter_equals_the_allocating_one(torch, eq, N, bc):
    for n, seed in ((16, 41), (9, 42)):  # the second call on a smaller mesh
        S, u = _solver(eq, N, n, bc, seed)
        ref, fref, out, flags = _both(torch, S, u)
        assert int(fref.sum()) > 0
        assert torch.equal(flags, fref)
        assert torch.equal(out, ref)
        allm = torch.ones(S.K, dtype=torch.uint8, device="cuda")
        ref, fref, out, flags = _both(torch, S, u, mask=allm)
        assert torch.equal(flags, fref) and torch.equal(out, ref)


def test_noalloc_limiter_rejects_meshes_beyond_its_scratch(torch):
    from paper_2106_06280_amd import binding
    v, t = inputs.jittered_mesh(420, seed=1)  # 352,800 P2 Euler elements: 68.9 MB of scratch
    S = binding.Solver(1, 2)
    S.mesh_upload(v, t, BC_TRANSMISSIVE, (1.0, 1.0))
    u = S.project_fn(inputs.UniformFlow(1.0, 0.1, 0.0, 1.0))
    out = torch.empty_like(u)
    flags = torch.empty(S.K, dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.CswdgError) as ei:
        S.csweno_limit_noalloc(u, out, flags)
    assert "too large" in str(ei.value)
