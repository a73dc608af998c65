"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host connectivity builder agrees bit for bit with the oracle's."""
import os
import re

import numpy as np
import pytest

from oracle.mesh import BC_PERIODIC, BC_TRANSMISSIVE, connectivity
from paper_2106_06280_amd import binding, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "cswdg.h")).read()
    return sorted(set(re.findall(r"\b(cswdg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    syms = _declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(binding._SIGS), set(syms) ^ set(binding._SIGS)


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (5, 3), (17, 4)])
@pytest.mark.parametrize("bc,period", [(BC_PERIODIC, (4.0, 2.0)), (BC_TRANSMISSIVE, (4.0, 2.0)),
                                       (BC_PERIODIC, (4.0, 0.0)), (BC_PERIODIC, (0.0, 2.0))])
def test_host_connectivity_bit_exact(n, seed, bc, period):
    v, t = inputs.jittered_mesh(n, -1.0, 3.0, 0.0, 2.0, seed=seed)
    t2 = t.copy()
    t2[1::4, 1], t2[1::4, 2] = t[1::4, 2], t[1::4, 1]  # some clockwise triangles
    tc, nbr, info = binding.host_connectivity(v, t2, bc, period)
    otri, onbr, oinfo = connectivity(v, t2, bc, period)
    assert np.array_equal(tc, otri.astype(np.int32))
    assert np.array_equal(nbr, onbr)
    assert np.array_equal(info, oinfo)


def test_mesh_size_limit():
    """More triangles than 32-bit [3][K] indices allow are rejected before
    any array is read (the arrays passed are tiny)."""
    vxy = np.zeros((3, 2))
    tri = np.zeros((1, 3), np.int32)
    out = np.zeros((1, 3), np.int32)
    info = np.zeros((1, 3), np.uint8)
    lim = binding.lib()
    rc = lim.cswdg_host_connectivity(3, vxy.ctypes.data, 715827883, tri.ctypes.data, 1, 0.0, 0.0, out.ctypes.data,
                                     out.ctypes.data, info.ctypes.data)
    assert rc == -1
    assert b"715,827,882" in lim.cswdg_last_error(None)


def test_host_connectivity_errors():
    v, t = inputs.jittered_mesh(3, seed=1)
    bad = t.copy()
    bad[0, 2] = bad[0, 1]
    with pytest.raises(binding.CswdgError) as ei:
        binding.host_connectivity(v, bad, BC_TRANSMISSIVE)
    assert ei.value.code == -2
    with pytest.raises(binding.CswdgError) as ei:
        binding.host_connectivity(v, t, BC_PERIODIC, (1.5, 1.0))
    assert ei.value.code == -2
    with pytest.raises(binding.CswdgError) as ei:
        binding.host_connectivity(v, t, 7, (1.0, 1.0))
    assert ei.value.code == -1
    dup = np.concatenate([t, t[:1]], axis=0)
    with pytest.raises(binding.CswdgError):
        binding.host_connectivity(v, dup, BC_TRANSMISSIVE)


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(ImportError):
        binding.lib()


@pytest.mark.parametrize("kind", ["periodic", "transmissive", "oneway", "ffstep"])
def test_host_tvb_decomposition_matches_the_oracle(kind):
    """The library's TVB midpoint decomposition (built on the host at mesh
    upload) against the oracle's: the same pair of neighbours per midpoint
    and the same coefficients up to rounding."""
    from oracle import tvb
    from oracle.dg import DG
    from oracle.mesh import Mesh
    if kind == "ffstep":
        v, t = inputs.forward_step_mesh(10, seed=4)
        bc, period = BC_TRANSMISSIVE, (0.0, 0.0)
    else:
        v, t = inputs.jittered_mesh(9, -1.0, 3.0, 0.0, 2.0, seed=6)
        bc, period = {"periodic": (BC_PERIODIC, (4.0, 2.0)), "transmissive": (BC_TRANSMISSIVE, (0.0, 0.0)),
                      "oneway": (BC_PERIODIC, (4.0, 0.0))}[kind]
    A, neg = binding.host_tvb_decomposition(v, t, bc, period)
    M = Mesh(v, t, bc, period)
    Ao = tvb.decomposition(DG(M, 1, 1))
    assert neg == 0
    assert np.array_equal(A != 0.0, Ao != 0.0)
    assert np.abs(A - Ao).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_host_tvb_decomposition_on_distorted_meshes(seed):
    """Interior vertices moved by up to 0.4 h: the library's and the
    oracle's decompositions still agree, and every midpoint still has a pair
    of nonnegative coefficients (the fallback for midpoints without one is
    not reached on these meshes)."""
    from oracle import tvb
    from oracle.dg import DG
    from oracle.mesh import Mesh
    v, t = inputs.jittered_mesh(12, jitter=0.4, seed=seed)
    A, neg = binding.host_tvb_decomposition(v, t, BC_TRANSMISSIVE)
    Ao = tvb.decomposition(DG(Mesh(v, t, BC_TRANSMISSIVE), 1, 0))
    assert neg == 0 and Ao.min() >= 0.0
    assert np.array_equal(A != 0.0, Ao != 0.0)
    assert np.abs(A - Ao).max() < 1e-12


def test_header_is_plain_c(tmp_path):
    """include/cswdg.h compiles as strict C99 (no C++ or torch types cross
    the boundary)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text('#include "cswdg.h"\nint main(void) { cswdg_params p = {0}; (void)p; return 0; }\n')
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
