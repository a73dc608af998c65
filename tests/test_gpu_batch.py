"""Batched instances, graph capture and schedule autotuning (GPU).

A mesh holding several independent instances must advance every instance
exactly as a solver holding that instance alone does (same kernels per
element, per-instance dt from an exact max/min): the comparison is bit for
bit.  Graph replays must equal the same steps run eagerly, replay after
replay, with eager work and synchronisations in between."""
import numpy as np
import pytest

from paper_2106_06280_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _instances(eq, ns, seed):
    b = inputs.batch_instances(n_inst=len(ns), seed=seed, n_burgers=len(ns) if eq == 0 else 0)
    out = []
    for d, n in zip(b, ns):
        vxy, tri = inputs.jittered_mesh(n, seed=d["mesh_seed"])
        out.append((vxy, tri, d["bc"], d["ic"]))
    return out


def _singles(torch, eq, N, inst, limiter_mode=0, **kw):
    from paper_2106_06280_amd import binding
    sol, us = [], []
    for vxy, tri, bc, ic in inst:
        S = binding.Solver(eq, N, limiter_mode=limiter_mode, **kw)
        S.mesh_upload(vxy, tri, bc, (1.0, 1.0))
        sol.append(S)
        us.append(S.project_fn(ic))
    return sol, us


def _batch(torch, eq, N, inst, us, limiter_mode=0, **kw):
    from paper_2106_06280_amd import binding
    B = binding.Solver(eq, N, limiter_mode=limiter_mode, **kw)
    B.mesh_upload_batch([(v, t) for v, t, _, _ in inst], [bc for _, _, bc, _ in inst], (1.0, 1.0))
    return B, torch.cat(us, dim=2).contiguous()


CASES = [(0, 1, [5, 9, 4, 12]), (0, 2, [7, 3, 10]), (1, 2, [6, 11, 4, 8, 5]), (1, 3, [4, 7])]


@pytest.mark.parametrize("eq,N,ns", CASES)
def test_batch_equals_single_instances(torch, eq, N, ns):
    inst = _instances(eq, ns, seed=20 + N)
    sol, us = _singles(torch, eq, N, inst)
    B, ub = _batch(torch, eq, N, inst, us)
    off = B.instances()
    assert off.tolist() == np.concatenate([[0], np.cumsum([2 * n * n for n in ns])]).tolist()
    # per-instance dt = the single solvers' dt, bit for bit
    dtb = B.max_dt(ub)
    for i, S in enumerate(sol):
        assert torch.equal(dtb[i:i + 1], S.max_dt(us[i])), i
    for step in range(4):
        B.ssprk3_step(ub)
        for S, u in zip(sol, us):
            S.ssprk3_step(u)
        for i, u in enumerate(us):
            assert torch.equal(ub[:, :, off[i]:off[i + 1]], u), (step, i)
    # troubled cells were exercised
    assert B.troubled_stats()[0] > 0
    assert B.status() & 3 == 0


@pytest.mark.parametrize("eq,recon", [(0, 1), (1, 1), (1, 2), (0, 3), (1, 3)])
def test_batch_other_reconstructions(torch, eq, recon):
    """The type-I, type-II and mixed reconstructions on a disjoint-union
    batch (P2): every instance of the batch equals its own solver, bit for
    bit, over three steps."""
    inst = _instances(eq, [6, 9, 4], seed=41 + recon)
    sol, us = _singles(torch, eq, 2, inst, reconstruction=recon)
    B, ub = _batch(torch, eq, 2, inst, us, reconstruction=recon)
    off = B.instances()
    for step in range(3):
        B.ssprk3_step(ub)
        for S, u in zip(sol, us):
            S.ssprk3_step(u)
        for i, u in enumerate(us):
            assert torch.equal(ub[:, :, off[i]:off[i + 1]], u), (step, i)
    assert B.troubled_stats()[0] > 0
    assert B.status() & 3 == 0


def test_batch_mixed_boundary_conditions(torch):
    """Periodic and transmissive instances in one mesh (Burgers, P2)."""
    inst = _instances(0, [6, 5, 8], seed=31)
    inst = [(v, t, bc, ic) for (v, t, _, ic), bc in zip(inst, [0, 1, 0])]
    sol, us = _singles(torch, 0, 2, inst)
    B, ub = _batch(torch, 0, 2, inst, us)
    off = B.instances()
    for _ in range(3):
        B.ssprk3_step(ub)
        for S, u in zip(sol, us):
            S.ssprk3_step(u)
    for i, u in enumerate(us):
        assert torch.equal(ub[:, :, off[i]:off[i + 1]], u), i


def test_graph_replays_equal_eager_steps(torch):
    """One graph holding 3 steps of a Burgers batch and an Euler batch;
    three replays, each checked against the same steps run eagerly on copies,
    with eager calls on the graph's solvers between replays."""
    from paper_2106_06280_amd import binding
    ib = _instances(0, [6, 9, 4], seed=41)
    ie = _instances(1, [5, 8, 7], seed=42)
    _, usb = _singles(torch, 0, 2, ib)
    _, use = _singles(torch, 1, 2, ie)
    Bb, ub = _batch(torch, 0, 2, ib, usb)
    Be, ue = _batch(torch, 1, 2, ie, use)
    # eager twins on separate solvers
    Rb, rb = _batch(torch, 0, 2, ib, usb)
    Re, re = _batch(torch, 1, 2, ie, use)
    g = binding.Graph([Bb, Be], [ub, ue], nsteps=3)
    assert g.nodes() > 0
    scratch = torch.empty_like(ue)
    for rep in range(3):
        g.launch()
        for _ in range(3):
            Rb.ssprk3_step(rb)
            Re.ssprk3_step(re)
        torch.cuda.synchronize()
        assert torch.equal(ub, rb), rep
        assert torch.equal(ue, re), rep
        # eager work on the graph's own solvers between replays (their scratch
        # buffers are shared with the graph)
        Be.dg_residual(ue, scratch)
        Bb.kxrcf(ub)
        torch.cuda.synchronize()
    assert Bb.status() & 3 == 0 and Be.status() & 3 == 0


def test_graph_single_solver_limiter_all(torch):
    from paper_2106_06280_amd import binding
    inst = _instances(1, [7], seed=51)
    sol, us = _singles(torch, 1, 2, inst, limiter_mode=1)
    S, u = sol[0], us[0]
    _, v = _singles(torch, 1, 2, inst, limiter_mode=1)
    R = _singles(torch, 1, 2, inst, limiter_mode=1)[0][0]
    v = v[0]
    g = binding.Graph([S], [u], nsteps=2)
    for rep in range(2):
        g.launch()
        R.ssprk3_step(v)
        R.ssprk3_step(v)
        torch.cuda.synchronize()
        assert torch.equal(u, v), rep


def test_autotune_picks_a_valid_schedule(torch):
    inst = _instances(1, [40], seed=61)
    sol, us = _singles(torch, 1, 2, inst)
    S, u = sol[0], us[0]
    r0 = S.dg_residual(u).clone()
    best, times = S.autotune(u, reps=3)
    assert len(times) == 30 and all(t > 0 for t in times.values())
    assert best in times and times[best] == min(times.values())
    assert S.get_schedule() == best
    r1 = S.dg_residual(u)
    scale = torch.max(torch.abs(r0)).item()
    assert torch.max(torch.abs(r1 - r0)).item() <= 1e-12 * scale
    # block size and block order do not change a single bit
    for b in (64, 128, 256):
        for x in (0, 1):
            S.set_schedule(best[0], b, x)
            assert torch.equal(S.dg_residual(u), r1), (b, x)


def test_adjoint_rejects_batched_mesh(torch):
    from paper_2106_06280_amd import binding
    inst = _instances(1, [4, 5], seed=71)
    _, us = _singles(torch, 1, 2, inst)
    B, ub = _batch(torch, 1, 2, inst, us)
    with pytest.raises(binding.CswdgError) as ei:
        B.dg_residual_vjp(ub, ub.clone())
    assert ei.value.code == -1
