"""Thin ctypes binding of libcswdg.so (include/cswdg.h).

Argument marshalling only: torch tensors supply device memory and the
stream; every step of the computation runs in the library's kernels.  The
binding raises if the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcswdg.so")

EQ_BURGERS, EQ_EULER = 0, 1
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
LIMIT_KXRCF, LIMIT_ALL, LIMIT_NONE = 0, 1, 2
INDICATOR_KXRCF, INDICATOR_TVB = 0, 1
STATUS_NONFINITE, STATUS_NEGATIVE, STATUS_RANK, STATUS_FOOT, STATUS_SCALED = 1, 2, 4, 8, 16

_lib = None


class CswdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cswdg error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("equation", ctypes.c_int), ("degree", ctypes.c_int), ("precision", ctypes.c_int),
                ("limiter_mode", ctypes.c_int), ("gas_gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("c_k", ctypes.c_double), ("eps_weno", ctypes.c_double), ("kxrcf_norm", ctypes.c_int),
                ("char_mode", ctypes.c_int), ("weights_mode", ctypes.c_int), ("positivity", ctypes.c_int),
                ("lf_mode", ctypes.c_int), ("p2_top", ctypes.c_int), ("indicator", ctypes.c_int),
                ("tvb_m", ctypes.c_double), ("gamma_mode", ctypes.c_int), ("ghost_mode", ctypes.c_int),
                ("reconstruction", ctypes.c_int), ("beta_mode", ctypes.c_int)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SIGS = {
    "cswdg_create": (ctypes.c_int, [ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]),
    "cswdg_destroy": (ctypes.c_int, [_P]),
    "cswdg_last_error": (ctypes.c_char_p, [_P]),
    "cswdg_mesh_upload": (ctypes.c_int, [_P, _I64, _P, _I64, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
    "cswdg_mesh_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "cswdg_host_connectivity": (ctypes.c_int, [_I64, _P, _I64, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "cswdg_host_tvb_decomposition": (ctypes.c_int, [_I64, _P, _I64, _P, ctypes.c_int, ctypes.c_double,
                                                    ctypes.c_double, _P, ctypes.POINTER(_I64)]),
    "cswdg_connectivity": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_stencil": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_int32)]),
    "cswdg_ic_points": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "cswdg_project": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_dg_residual": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_max_dt": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_kxrcf": (ctypes.c_int, [_P, _P, _P, _P]),
    "cswdg_csweno_limit": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "cswdg_csweno_limit_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "cswdg_rk_stage": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
    "cswdg_ssprk3_step": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_last_dt": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "cswdg_troubled_count": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "cswdg_status": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32)]),
    "cswdg_troubled_stats": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.c_int]),
    "cswdg_dg_residual_vjp": (ctypes.c_int, [_P, _P, _P, _P]),
    "cswdg_csweno_limit_vjp": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "cswdg_tape_bytes": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "cswdg_ssprk3_step_tape": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int]),
    "cswdg_ssprk3_step_vjp": (ctypes.c_int, [_P, _P, _P, _P]),
    "cswdg_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "cswdg_profile_select": (ctypes.c_int, [_P, ctypes.c_uint32]),
    "cswdg_set_boundary": (ctypes.c_int, [_P, _P, _P]),
    "cswdg_positivity": (ctypes.c_int, [_P, _P]),
    "cswdg_set_moving_shock": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double]),
    "cswdg_set_time": (ctypes.c_int, [_P, ctypes.c_double]),
    "cswdg_time": (ctypes.c_int, [_P, _P]),
    "cswdg_kernel_times": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "cswdg_mesh_upload_batch": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_double]),
    "cswdg_instances": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    "cswdg_set_schedule": (ctypes.c_int, [_P, _P]),
    "cswdg_get_schedule": (ctypes.c_int, [_P, _P]),
    "cswdg_autotune": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_int32)]),
    "cswdg_graph_capture": (ctypes.c_int, [ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.POINTER(_P)]),
    "cswdg_graph_launch": (ctypes.c_int, [_P, _P]),
    "cswdg_graph_nodes": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "cswdg_graph_destroy": (ctypes.c_int, [_P]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python paper_2106_06280_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != 0:
        msg = lib().cswdg_last_error(handle)
        raise CswdgError(rc, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def host_connectivity(vxy, tri, bc, period=(0.0, 0.0)):
    """Host-only connectivity builder: (tri_ccw, nbr, info) as numpy arrays."""
    vxy = np.ascontiguousarray(vxy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    K = tri.shape[0]
    tc = np.zeros((K, 3), np.int32)
    nbr = np.zeros((K, 3), np.int32)
    info = np.zeros((K, 3), np.uint8)
    rc = lib().cswdg_host_connectivity(vxy.shape[0], vxy.ctypes.data, K, tri.ctypes.data, bc,
                                       float(period[0]), float(period[1]), tc.ctypes.data,
                                       nbr.ctypes.data, info.ctypes.data)
    _check(rc, None)
    return tc, nbr, info


def host_tvb_decomposition(vxy, tri, bc, period=(0.0, 0.0)):
    """Host-only builder of the TVB indicator's midpoint decomposition:
    (A [K, 3, 3], number of midpoints without a nonnegative pair)."""
    vxy = np.ascontiguousarray(vxy, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    K = tri.shape[0]
    A = np.zeros((K, 3, 3), np.float64)
    neg = _I64(0)
    rc = lib().cswdg_host_tvb_decomposition(vxy.shape[0], vxy.ctypes.data, K, tri.ctypes.data, bc,
                                            float(period[0]), float(period[1]), A.ctypes.data, ctypes.byref(neg))
    _check(rc, None)
    return A, int(neg.value)


# p2_top values (Section 3.2, Steps 1-2 for P2: the fourth member of the
# N >= 2 hierarchy) and the oracle's name of each reading
TOP_DEFAULT, TOP_QUADRATIC, TOP_QUARTIC, TOP_CUBIC_TEL, TOP_CUBIC, TOP_SEXTIC = 0, 1, 2, 3, 4, 5
# reconstruction values: the paper's hierarchical WENO, type-I, type-II or
# mixed WENO
RECON_HIERARCHICAL, RECON_TYPE1, RECON_TYPE2, RECON_MIXED = 0, 1, 2, 3
TOP_NAMES = {TOP_QUADRATIC: "quadratic", TOP_QUARTIC: "quartic", TOP_CUBIC_TEL: "cubic_tel", TOP_CUBIC: "cubic",
             TOP_SEXTIC: "sextic"}


def top_name(degree, p2_top):
    """The reading a p2_top value selects for degree N (None: N = 1, whose
    hierarchy has the quadratic q_3 on top)."""
    if degree == 1:
        return None
    if p2_top == TOP_DEFAULT:
        return "quadratic" if degree == 2 else "quartic"
    return TOP_NAMES[p2_top]


class Solver:
    """One solver = one equation, degree and mesh on the current GPU."""

    def __init__(self, equation, degree, limiter_mode=LIMIT_KXRCF, precision=0, gamma=1.4, cfl=0.0,
                 c_k=0.0, eps=0.0, stream=None, kxrcf_norm=0, char_mode=0, weights_mode=0, positivity=0,
                 lf_mode=0, p2_top=0, indicator=INDICATOR_KXRCF, tvb_m=0.0, gamma_mode=0, ghost_mode=0,
                 reconstruction=0, beta_mode=0):
        import torch
        self.torch = torch
        p = Params(equation, degree, precision, limiter_mode, gamma, cfl, c_k, eps, kxrcf_norm, char_mode,
                   weights_mode, positivity, lf_mode, p2_top, indicator, tvb_m, gamma_mode, ghost_mode, reconstruction,
                   beta_mode)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().cswdg_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), None)
        self.h = h
        self.equation, self.degree, self.precision = equation, degree, precision
        self.dtype = torch.float32 if precision == 1 else torch.float64
        self.m = 1 if equation == EQ_BURGERS else 4
        self.Np = (degree + 1) * (degree + 2) // 2
        self.K = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().cswdg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _c(self, rc):
        _check(rc, self.h)

    # -- argument checks (the C ABI takes raw pointers and cannot check sizes) --
    def _n_inst(self):
        if not hasattr(self, "_ninst"):
            self._ninst = len(self.instances()) - 1
        return self._ninst

    def _dev(self, t, name, shape, dtype):
        if t is None:
            raise ValueError(f"{name} is required")
        if not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name}: expected a contiguous CUDA tensor {tuple(shape)} {dtype}, "
                             f"got {tuple(t.shape)} {t.dtype} (cuda={t.is_cuda}, contiguous={t.is_contiguous()})")
        return t

    def _st(self, t, name="state"):
        return self._dev(t, name, (self.m, self.Np, self.K), self.dtype)

    def _dt(self, t, name="dt"):
        return self._dev(t, name, (self._n_inst(),), self.torch.float64)

    def _mask(self, m):
        if m is None:
            return None
        m = m.to(device="cuda", dtype=self.torch.uint8).contiguous()
        return self._dev(m, "mask", (self.K,), self.torch.uint8)

    # -- mesh ------------------------------------------------------------
    def mesh_upload(self, vxy, tri, bc, period=(0.0, 0.0)):
        vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._c(lib().cswdg_mesh_upload(self.h, vxy.shape[0], vxy.ctypes.data, tri.shape[0], tri.ctypes.data,
                                        bc, float(period[0]), float(period[1])))
        self.K = tri.shape[0]
        self.__dict__.pop("_ninst", None)

    def mesh_upload_batch(self, meshes, bcs, period=(1.0, 1.0)):
        """meshes: list of (vxy [nv][2], tri [nt][3]) with instance-local vertex
        ids; bcs: one boundary condition per instance."""
        nv = np.array([m[0].shape[0] for m in meshes], np.int64)
        nt = np.array([m[1].shape[0] for m in meshes], np.int64)
        vxy = np.ascontiguousarray(np.concatenate([np.asarray(m[0], np.float64) for m in meshes]))
        tri = np.ascontiguousarray(np.concatenate([np.asarray(m[1], np.int32) for m in meshes]))
        bc = np.ascontiguousarray(np.asarray(bcs, np.int32))
        if bc.shape != (len(meshes),):
            raise ValueError("one boundary condition per instance")
        self._c(lib().cswdg_mesh_upload_batch(self.h, len(meshes), nv.ctypes.data, vxy.ctypes.data, nt.ctypes.data,
                                              tri.ctypes.data, bc.ctypes.data, float(period[0]), float(period[1])))
        self.K = int(nt.sum())
        self.__dict__.pop("_ninst", None)

    def set_boundary(self, kinds=None, inflow=None):
        """kinds [K, 3] (0 outflow, 1 wall, 2 inflow; read on boundary faces);
        inflow: conserved state [m] of inflow faces."""
        k = None
        if kinds is not None:
            k = np.ascontiguousarray(np.asarray(kinds, dtype=np.uint8))
            if k.shape != (self.K, 3):
                raise ValueError(f"kinds: expected ({self.K}, 3), got {k.shape}")
        s = None
        if inflow is not None:
            s = np.ascontiguousarray(np.asarray(inflow, dtype=np.float64))
            if s.shape != (self.m,):
                raise ValueError(f"inflow: expected ({self.m},), got {s.shape}")
        self._c(lib().cswdg_set_boundary(self.h, None if k is None else k.ctypes.data,
                                         None if s is None else s.ctypes.data))

    def set_moving_shock(self, post, pre, n, d0, speed):
        """The planar shock of boundary kind 3: post where n.x < d0 + speed t
        (conserved states [4]); see cswdg_set_moving_shock."""
        a = np.ascontiguousarray(np.asarray(post, dtype=np.float64))
        b = np.ascontiguousarray(np.asarray(pre, dtype=np.float64))
        if a.shape != (4,) or b.shape != (4,):
            raise ValueError("moving shock: post and pre are [4] conserved states")
        self._c(lib().cswdg_set_moving_shock(self.h, a.ctypes.data, b.ctypes.data, float(n[0]), float(n[1]),
                                             float(d0), float(speed)))

    def set_time(self, t):
        self._c(lib().cswdg_set_time(self.h, float(t)))

    def time(self):
        """Solution time of each instance (numpy float64 [n_inst])."""
        out = np.zeros(self._n_inst(), np.float64)
        self._c(lib().cswdg_time(self.h, out.ctypes.data))
        return out

    def instances(self):
        """Instance offsets (numpy int64 [n_inst + 1])."""
        n = ctypes.c_int32()
        self._c(lib().cswdg_instances(self.h, ctypes.byref(n), None))
        off = np.zeros(n.value + 1, np.int64)
        self._c(lib().cswdg_instances(self.h, ctypes.byref(n), off.ctypes.data))
        return off

    def mesh_info(self):
        k, f = _I64(), _I64()
        self._c(lib().cswdg_mesh_info(self.h, ctypes.byref(k), ctypes.byref(f)))
        return k.value, f.value

    def connectivity(self):
        nbr = np.zeros((self.K, 3), np.int32)
        info = np.zeros((self.K, 3), np.uint8)
        self._c(lib().cswdg_connectivity(self.h, nbr.ctypes.data, info.ctypes.data))
        return nbr, info

    def stencil(self, e):
        ids = np.zeros(12, np.int32)
        n = ctypes.c_int32()
        self._c(lib().cswdg_stencil(self.h, int(e), ids.ctypes.data, ctypes.byref(n)))
        return ids[: n.value].tolist()

    # -- state helpers ----------------------------------------------------
    def empty_state(self):
        return self.torch.empty((self.m, self.Np, self.K), dtype=self.dtype, device="cuda")

    def to_device(self, u_kmn):
        """Oracle layout [K, m, Np] (numpy) -> device layout [m, Np, K]."""
        a = np.ascontiguousarray(np.transpose(np.asarray(u_kmn, dtype=np.float64), (1, 2, 0)))
        return self.torch.from_numpy(a).to(device="cuda", dtype=self.dtype)

    @staticmethod
    def to_host(u):
        """Device layout [m, Np, K] -> numpy [K, m, Np]."""
        return np.ascontiguousarray(np.transpose(u.detach().double().cpu().numpy(), (2, 0, 1)))

    def ic_points(self):
        nq = ctypes.c_int32()
        self._c(lib().cswdg_ic_points(self.h, None, ctypes.byref(nq)))
        xy = self.torch.empty((2, nq.value, self.K), dtype=self.torch.float64, device="cuda")
        self._c(lib().cswdg_ic_points(self.h, _ptr(xy), ctypes.byref(nq)))
        return xy

    def project(self, vals):
        """vals [m, nq, K] device double -> coefficients."""
        nq = ctypes.c_int32()
        self._c(lib().cswdg_ic_points(self.h, None, ctypes.byref(nq)))
        vals = self._dev(vals.contiguous(), "vals", (self.m, nq.value, self.K), self.torch.float64)
        u = self.empty_state()
        self._c(lib().cswdg_project(self.h, _ptr(vals), _ptr(u)))
        return u

    def project_fn(self, fn):
        """Evaluate fn(x, y) (numpy, pointwise) at the projection points and project."""
        xy = self.ic_points().cpu().numpy()
        v = np.asarray(fn(xy[0], xy[1]), dtype=np.float64)
        if v.ndim == 2:
            v = v[None]
        else:
            v = np.moveaxis(v, -1, 0)
        if v.shape[0] != self.m:
            raise ValueError(f"fn returns {v.shape[0]} variable(s); this solver has {self.m}")
        return self.project(self.torch.from_numpy(np.ascontiguousarray(v)).to("cuda"))

    # -- operators --------------------------------------------------------
    def dg_residual(self, u, r=None):
        if r is None:
            r = self.empty_state()
        self._st(u, "u")
        self._st(r, "r")
        self._c(lib().cswdg_dg_residual(self.h, _ptr(u), _ptr(r)))
        return r

    def max_dt(self, u, dt=None):
        if dt is None:
            dt = self.torch.zeros(self._n_inst(), dtype=self.torch.float64, device="cuda")
        self._st(u, "u")
        self._dt(dt)
        self._c(lib().cswdg_max_dt(self.h, _ptr(u), _ptr(dt)))
        return dt

    def kxrcf(self, u, want_R=True):
        flags = self.torch.zeros(self.K, dtype=self.torch.uint8, device="cuda")
        R = self.torch.zeros(self.K, dtype=self.torch.float64, device="cuda") if want_R else None
        self._st(u, "u")
        self._c(lib().cswdg_kxrcf(self.h, _ptr(u), _ptr(flags), _ptr(R)))
        return flags, R

    def csweno_limit(self, u_in, u_out=None, mask=None):
        if u_out is None:
            u_out = self.empty_state()
        flags = self.torch.zeros(self.K, dtype=self.torch.uint8, device="cuda")
        m = self._mask(mask)
        self._st(u_in, "u_in")
        self._st(u_out, "u_out")
        self._c(lib().cswdg_csweno_limit(self.h, _ptr(u_in), _ptr(u_out), _ptr(flags), _ptr(m)))
        return u_out, flags

    def csweno_limit_noalloc(self, u_in, u_out, flags, mask=None):
        """cswdg_csweno_limit_noalloc: u_out and flags (device uint8 [K])
        are the caller's; the library allocates nothing."""
        m = self._mask(mask)
        self._st(u_in, "u_in")
        self._st(u_out, "u_out")
        self._dev(flags, "flags", (self.K,), self.torch.uint8)
        self._c(lib().cswdg_csweno_limit_noalloc(self.h, _ptr(u_in), _ptr(u_out), _ptr(flags), _ptr(m)))
        return u_out, flags

    def rk_stage(self, stage, u_n, u_prev, out, dt):
        if int(stage) > 1:
            self._st(u_n, "u_n")
        self._st(u_prev, "u_prev")
        self._st(out, "out")
        self._dt(dt)
        self._c(lib().cswdg_rk_stage(self.h, int(stage), _ptr(u_n), _ptr(u_prev), _ptr(out), _ptr(dt)))
        return out

    def positivity(self, u):
        """Positivity-preserving scaling of an Euler state in place (not part
        of the paper's method; see cswdg_positivity)."""
        self._st(u, "u")
        self._c(lib().cswdg_positivity(self.h, _ptr(u)))
        return u

    def ssprk3_step(self, u, dt=None):
        self._st(u, "u")
        if dt is not None:
            self._dt(dt)
        self._c(lib().cswdg_ssprk3_step(self.h, _ptr(u), _ptr(dt)))
        return u

    # -- adjoint ------------------------------------------------------------
    def dg_residual_vjp(self, u, r_bar, u_bar=None):
        if u_bar is None:
            u_bar = self.empty_state()
        self._st(u, "u")
        self._st(r_bar, "r_bar")
        self._st(u_bar, "u_bar")
        self._c(lib().cswdg_dg_residual_vjp(self.h, _ptr(u), _ptr(r_bar), _ptr(u_bar)))
        return u_bar

    def csweno_limit_vjp(self, w, y_bar, mask=None, w_bar=None):
        if w_bar is None:
            w_bar = self.empty_state()
        m = self._mask(mask)
        self._st(w, "w")
        self._st(y_bar, "y_bar")
        self._st(w_bar, "w_bar")
        self._c(lib().cswdg_csweno_limit_vjp(self.h, _ptr(w), _ptr(m), _ptr(y_bar), _ptr(w_bar)))
        return w_bar

    def new_tape(self):
        n = _I64()
        self._c(lib().cswdg_tape_bytes(self.h, ctypes.byref(n)))
        return self.torch.empty(n.value, dtype=self.torch.uint8, device="cuda")

    def tape_dt(self, tape):
        """dt stored in a tape (device tensor view)."""
        n = tape.numel()
        return tape[n - 256:n - 248].view(self.torch.float64)

    def _tape(self, tape):
        n = _I64()
        self._c(lib().cswdg_tape_bytes(self.h, ctypes.byref(n)))
        return self._dev(tape, "tape", (n.value,), self.torch.uint8)

    def ssprk3_step_tape(self, u, tape, dt=None, replay=False):
        self._st(u, "u")
        self._tape(tape)
        if dt is not None:
            self._dt(dt)
        self._c(lib().cswdg_ssprk3_step_tape(self.h, _ptr(u), _ptr(dt), _ptr(tape), 1 if replay else 0))
        return u

    def ssprk3_step_vjp(self, tape, y_bar, u_bar=None):
        if u_bar is None:
            u_bar = self.empty_state()
        self._tape(tape)
        self._st(y_bar, "y_bar")
        self._st(u_bar, "u_bar")
        self._c(lib().cswdg_ssprk3_step_vjp(self.h, _ptr(tape), _ptr(y_bar), _ptr(u_bar)))
        return u_bar

    def last_dt_ptr(self):
        p = ctypes.c_void_p()
        self._c(lib().cswdg_last_dt(self.h, ctypes.byref(p)))
        return p.value

    def troubled_count(self):
        c = _I64()
        self._c(lib().cswdg_troubled_count(self.h, ctypes.byref(c)))
        return c.value

    def troubled_stats(self, reset=False):
        t, c = _I64(), _I64()
        self._c(lib().cswdg_troubled_stats(self.h, ctypes.byref(t), ctypes.byref(c), 1 if reset else 0))
        return t.value, c.value

    def status(self):
        v = ctypes.c_uint32()
        self._c(lib().cswdg_status(self.h, ctypes.byref(v)))
        return v.value

    # -- schedules and autotuning --------------------------------------------
    def set_schedule(self, variant, block, xcd):
        a = np.array([variant, block, xcd], np.int32)
        self._c(lib().cswdg_set_schedule(self.h, a.ctypes.data))

    def get_schedule(self):
        a = np.zeros(3, np.int32)
        self._c(lib().cswdg_get_schedule(self.h, a.ctypes.data))
        return tuple(int(x) for x in a)

    def autotune(self, u, reps=5):
        """Time every residual schedule on u; keep the fastest.  Returns
        (schedule, {schedule: microseconds})."""
        a = np.zeros(3, np.int32)
        t = np.zeros(30, np.float64)
        n = ctypes.c_int32()
        self._st(u, "u")
        self._c(lib().cswdg_autotune(self.h, _ptr(u), int(reps), a.ctypes.data, t.ctypes.data, ctypes.byref(n)))
        cands = [(v, b, x) for v in (0, 1, 2, 3, 4) for b in (64, 128, 256) for x in (0, 1)]
        return tuple(int(x) for x in a), {c: float(t[i]) for i, c in enumerate(cands[: n.value])}

    KERNEL_CLASSES = ("residual_rk", "max_dt", "kxrcf", "compact_mask", "limiter", "scatter", "copy", "zero",
                      "project", "residual_vjp", "limiter_vjp", "positivity")

    def profile(self, enable=True, only=None):
        """HIP-event timing of every launch (or only of the named kernel
        classes) until profile(False)."""
        mask = 0xFFFFFFFF if only is None else sum(1 << self.KERNEL_CLASSES.index(k) for k in only)
        self._c(lib().cswdg_profile_select(self.h, mask))
        self._c(lib().cswdg_profile(self.h, 1 if enable else 0))

    def kernel_times(self):
        cap = 16
        names = (ctypes.c_char_p * cap)()
        tot = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        n = ctypes.c_int()
        self._c(lib().cswdg_kernel_times(self.h, names, tot, cnt, cap, ctypes.byref(n)))
        return {names[i].decode(): (tot[i], cnt[i]) for i in range(min(n.value, cap))}


class Graph:
    """nsteps SSP-RK3 steps of several solvers, each on its own state, recorded
    into one HIP graph; launch() advances every state by nsteps steps."""

    def __init__(self, solvers, states, nsteps):
        import torch
        self.torch = torch
        self.solvers = list(solvers)
        self.states = list(states)  # kept alive: the graph holds their addresses
        for s, u in zip(self.solvers, self.states):
            if not u.is_contiguous() or tuple(u.shape) != (s.m, s.Np, s.K):
                raise ValueError("state must be a contiguous [m, Np, K] tensor of its solver")
        n = len(self.solvers)
        hs = (ctypes.c_void_p * n)(*[s.h.value for s in self.solvers])
        us = (ctypes.c_void_p * n)(*[u.data_ptr() for u in self.states])
        g = ctypes.c_void_p()
        _check(lib().cswdg_graph_capture(n, hs, us, int(nsteps), ctypes.byref(g)), None)
        self.g = g
        self.nsteps = nsteps

    def launch(self, stream=None):
        if stream is None:
            stream = self.torch.cuda.current_stream()
        _check(lib().cswdg_graph_launch(self.g, ctypes.c_void_p(stream.cuda_stream)), None)

    def nodes(self):
        n = _I64()
        _check(lib().cswdg_graph_nodes(self.g, ctypes.byref(n)), None)
        return n.value

    def __del__(self):
        try:
            if getattr(self, "g", None):
                lib().cswdg_graph_destroy(self.g)
                self.g = None
        except Exception:
            pass
