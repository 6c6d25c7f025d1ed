"""ctypes binding of libvofl (include/vofl.h): argument marshalling only.

Every computation runs in the HIP kernels of libvofl.so. PyTorch supplies
device memory (tensor.data_ptr()) and the stream
(torch.cuda.current_stream().cuda_stream). Importing this module does not
touch the GPU; loading the library raises if libvofl.so has not been built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvofl.so")

VOFL_OK = 0
VOFL_ERR_INVALID = -1
VOFL_ERR_NOMEM = -2
VOFL_ERR_DEVICE = -3
VOFL_ERR_UNSTABLE = -4
VOFL_ERR_UNSUPPORTED = -5
VOFL_FP64 = 0
VOFL_FP32 = 1
VOFL_MODEL_SEISMIC = 0
VOFL_MODEL_GENERIC = 1
VOFL_PROBE_READ = 0
VOFL_PROBE_WRITE = 1
VOFL_PROBE_COPY = 2
VOFL_PROBE_NONTEMPORAL = 1
VOFL_PROBE_DEEP = 2
VOFL_OP_S1 = 1
VOFL_OP_S2 = 2

# every function declared in include/vofl.h
ABI_FUNCTIONS = (
    "vofl_plan", "vofl_plan_footprint", "vofl_apply", "vofl_step", "vofl_step_graph", "vofl_solve",
    "vofl_step_begin", "vofl_step_advance", "vofl_step_end", "vofl_lffp_start", "vofl_lffp_step",
    "vofl_cnfp_step", "vofl_step_batch", "vofl_sync_status", "vofl_set_timing", "vofl_kernel_times",
    "vofl_plan_info", "vofl_destroy", "vofl_last_error", "vofl_version", "vofl_apply_noalloc",
    "vofl_stream_probe",
)

_c_double_p = ctypes.POINTER(ctypes.c_double)


class vofl_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("model", ctypes.c_int),
        ("c0", ctypes.c_double),
        ("omega0", ctypes.c_double),
        ("Q", _c_double_p),
        ("gamma", _c_double_p),
        ("s", _c_double_p),
        ("kappa", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("M", ctypes.c_int),
        ("dt", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("max_batch", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("coef_per_solve", ctypes.c_int),
        ("hbm_budget", ctypes.c_size_t),
        ("tune_steps", ctypes.c_int),
        ("order", ctypes.c_int),
        ("c0_field", _c_double_p),
    ]


class VoflError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vofl error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libvofl.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libvofl.so not found at {LIB_PATH}; run "
                          "`python -m paper_2311_13049_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.vofl_plan.argtypes = [ctypes.POINTER(vofl_desc), vp, ctypes.POINTER(vp)]
    lib.vofl_plan_footprint.argtypes = [ctypes.POINTER(vofl_desc), ctypes.POINTER(ctypes.c_size_t)]
    lib.vofl_apply.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, vp]
    lib.vofl_step.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.vofl_step_graph.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.vofl_step_begin.argtypes = [vp, vp, vp, vp]
    lib.vofl_step_advance.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.vofl_step_end.argtypes = [vp, vp, vp, vp]
    lib.vofl_lffp_start.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.vofl_lffp_step.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.vofl_cnfp_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_longlong), vp]
    lib.vofl_solve.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp]
    lib.vofl_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int, vp]
    lib.vofl_sync_status.argtypes = [vp, vp]
    lib.vofl_set_timing.argtypes = [vp, ctypes.c_int]
    lib.vofl_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), _c_double_p,
                                      ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
    lib.vofl_plan_info.argtypes = [vp, _c_double_p, ctypes.c_int]
    lib.vofl_destroy.argtypes = [vp]
    lib.vofl_apply_noalloc.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, vp, ctypes.c_int,
                                       ctypes.c_int, vp, vp, ctypes.c_int, vp]
    lib.vofl_stream_probe.argtypes = [ctypes.c_int, vp, vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp]
    lib.vofl_last_error.restype = ctypes.c_char_p
    lib.vofl_version.restype = ctypes.c_char_p
    for name in ("vofl_plan", "vofl_plan_footprint", "vofl_apply", "vofl_step", "vofl_step_graph", "vofl_solve",
                 "vofl_step_begin", "vofl_step_advance", "vofl_step_end", "vofl_lffp_start", "vofl_lffp_step",
                 "vofl_cnfp_step",
                 "vofl_step_batch", "vofl_sync_status", "vofl_set_timing", "vofl_kernel_times",
                 "vofl_plan_info", "vofl_destroy", "vofl_apply_noalloc", "vofl_stream_probe"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        msg = load_library().vofl_last_error().decode()
        raise VoflError(rc, msg)
    return rc


def make_desc(shape, lo, hi, *, model="seismic", c0=1.0, omega0=1.0, Q=None, gamma=None,
              s=None, kappa=1.0, lam=0.0, M=8, dt=1e-3, precision="fp64", max_batch=1,
              batch=1, coef_per_solve=False, hbm_budget=0, tune_steps=0, order=2, c0_field=None):
    """Build a vofl_desc; returns (desc, keepalive) where keepalive holds the host arrays.
    c0_field: per-point phase velocities (layered media; replaces c0)."""
    shape = tuple(int(n) for n in shape)
    d = vofl_desc()
    d.ndim = len(shape)
    for i in range(3):
        d.n[i] = shape[i] if i < len(shape) else 1
        d.lo[i] = float(lo[i]) if i < len(shape) else 0.0
        d.hi[i] = float(hi[i]) if i < len(shape) else 1.0
    d.model = VOFL_MODEL_SEISMIC if model == "seismic" else VOFL_MODEL_GENERIC
    d.c0, d.omega0 = float(c0), float(omega0)
    keep = []

    def arr(x):
        if x is None:
            return None
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
        keep.append(a)
        return a.ctypes.data_as(_c_double_p)

    d.Q = arr(Q)
    d.gamma = arr(gamma)
    d.s = arr(s)
    d.kappa, d.lambda_ = float(kappa), float(lam)
    d.M = int(M)
    d.dt = float(dt)
    d.precision = VOFL_FP32 if precision in ("fp32", "float32", VOFL_FP32) else VOFL_FP64
    d.max_batch = int(max_batch)
    d.batch = int(batch)
    d.coef_per_solve = 1 if coef_per_solve else 0
    d.hbm_budget = int(hbm_budget)
    d.tune_steps = int(tune_steps)
    d.order = int(order)
    d.c0_field = arr(c0_field)
    return d, keep


# --- functions with the names of the C ABI ---------------------------------

def vofl_plan(desc: vofl_desc, stream=0) -> int:
    h = ctypes.c_void_p()
    _check(load_library().vofl_plan(ctypes.byref(desc), ctypes.c_void_p(stream), ctypes.byref(h)))
    return h.value


def vofl_plan_footprint(desc: vofl_desc) -> int:
    b = ctypes.c_size_t()
    _check(load_library().vofl_plan_footprint(ctypes.byref(desc), ctypes.byref(b)))
    return b.value


def vofl_apply(plan: int, op: int, u_ptr: int, out_ptr: int, nfields: int, stream=0) -> None:
    _check(load_library().vofl_apply(ctypes.c_void_p(plan), op, ctypes.c_void_p(u_ptr),
                                     ctypes.c_void_p(out_ptr), nfields, ctypes.c_void_p(stream)))


def vofl_step(plan: int, u_ptr: int, v_ptr: int, nsteps: int, stream=0) -> None:
    _check(load_library().vofl_step(ctypes.c_void_p(plan), ctypes.c_void_p(u_ptr),
                                    ctypes.c_void_p(v_ptr), nsteps, ctypes.c_void_p(stream)))


def vofl_step_graph(plan: int, u_ptr: int, v_ptr: int, nsteps: int, stream=0) -> None:
    _check(load_library().vofl_step_graph(ctypes.c_void_p(plan), ctypes.c_void_p(u_ptr),
                                          ctypes.c_void_p(v_ptr), nsteps, ctypes.c_void_p(stream)))


def vofl_apply_noalloc(n: int, lo: float, hi: float, s_ptr: int, M: int, precision: int, u_ptr: int,
                       out_ptr: int, nfields: int, stream=0) -> None:
    _check(load_library().vofl_apply_noalloc(int(n), float(lo), float(hi), ctypes.c_void_p(s_ptr), int(M),
                                             int(precision), ctypes.c_void_p(u_ptr), ctypes.c_void_p(out_ptr),
                                             int(nfields), ctypes.c_void_p(stream)))


def vofl_stream_probe(kind: int, src_ptr: int, dst_ptr: int, nbytes: int, blocks: int, flags: int = 0,
                      stream=0) -> None:
    _check(load_library().vofl_stream_probe(int(kind), ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr),
                                            int(nbytes), int(blocks), int(flags), ctypes.c_void_p(stream)))


def vofl_step_begin(plan: int, u_ptr: int, v_ptr: int, stream=0) -> None:
    _check(load_library().vofl_step_begin(ctypes.c_void_p(plan), ctypes.c_void_p(u_ptr),
                                          ctypes.c_void_p(v_ptr), ctypes.c_void_p(stream)))


def vofl_step_advance(plan: int, nsteps: int, use_graph: int = 0, stream=0) -> None:
    _check(load_library().vofl_step_advance(ctypes.c_void_p(plan), int(nsteps), int(use_graph),
                                            ctypes.c_void_p(stream)))


def vofl_step_end(plan: int, u_ptr: int, v_ptr: int, stream=0) -> None:
    _check(load_library().vofl_step_end(ctypes.c_void_p(plan), ctypes.c_void_p(u_ptr),
                                        ctypes.c_void_p(v_ptr), ctypes.c_void_p(stream)))


def vofl_lffp_start(plan: int, phi_ptr: int, psi_ptr: int, u_prev_ptr: int, u_ptr: int, stream=0) -> None:
    _check(load_library().vofl_lffp_start(ctypes.c_void_p(plan), ctypes.c_void_p(phi_ptr),
                                          ctypes.c_void_p(psi_ptr), ctypes.c_void_p(u_prev_ptr),
                                          ctypes.c_void_p(u_ptr), ctypes.c_void_p(stream)))


def vofl_lffp_step(plan: int, u_prev_ptr: int, u_ptr: int, nsteps: int, stream=0) -> None:
    _check(load_library().vofl_lffp_step(ctypes.c_void_p(plan), ctypes.c_void_p(u_prev_ptr),
                                         ctypes.c_void_p(u_ptr), nsteps, ctypes.c_void_p(stream)))


def vofl_cnfp_step(plan: int, u_prev_ptr: int, u_ptr: int, nsteps: int, tol: float, max_iter: int,
                   stream=0) -> int:
    it = ctypes.c_longlong(0)
    _check(load_library().vofl_cnfp_step(ctypes.c_void_p(plan), ctypes.c_void_p(u_prev_ptr),
                                         ctypes.c_void_p(u_ptr), nsteps, float(tol), int(max_iter),
                                         ctypes.byref(it), ctypes.c_void_p(stream)))
    return it.value


def vofl_solve(plan: int, u0_ptr: int, v0_ptr: int, nsteps: int, u_ptr: int, v_ptr: int,
               stream=0) -> None:
    _check(load_library().vofl_solve(ctypes.c_void_p(plan), ctypes.c_void_p(u0_ptr),
                                     ctypes.c_void_p(v0_ptr), nsteps, ctypes.c_void_p(u_ptr),
                                     ctypes.c_void_p(v_ptr), ctypes.c_void_p(stream)))


def vofl_step_batch(plans, u_ptrs, v_ptrs, nsteps, stream=0) -> None:
    n = len(plans)
    P = (ctypes.c_void_p * n)(*plans)
    U = (ctypes.c_void_p * n)(*u_ptrs)
    V = (ctypes.c_void_p * n)(*v_ptrs)
    S = (ctypes.c_int * n)(*nsteps)
    _check(load_library().vofl_step_batch(P, U, V, S, n, ctypes.c_void_p(stream)))


def vofl_sync_status(plan: int, stream=0) -> int:
    return load_library().vofl_sync_status(ctypes.c_void_p(plan), ctypes.c_void_p(stream))


def vofl_set_timing(plan: int, enable: bool) -> None:
    _check(load_library().vofl_set_timing(ctypes.c_void_p(plan), 1 if enable else 0))


def vofl_kernel_times(plan: int) -> dict:
    lib = load_library()
    cap = 64
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_longlong * cap)()
    k = _check(lib.vofl_kernel_times(ctypes.c_void_p(plan), names, ms, cnt, cap))
    return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(k, cap))}


def vofl_plan_info(plan: int) -> dict:
    out = (ctypes.c_double * 8)()
    _check(load_library().vofl_plan_info(ctypes.c_void_p(plan), out, 8))
    return dict(mean_order_offset=out[0], kappa0=out[1], beta0=out[2], N=int(out[3]),
                device_bytes=int(out[4]), c2r_variant=int(out[5]), mid_variant=int(out[6]),
                contig_variant=int(out[7]))


def vofl_destroy(plan: int) -> None:
    _check(load_library().vofl_destroy(ctypes.c_void_p(plan)))


def vofl_last_error() -> str:
    return load_library().vofl_last_error().decode()


def vofl_version() -> str:
    return load_library().vofl_version().decode()


# --- torch-facing convenience wrapper ---------------------------------------

class Plan:
    """A plan bound to torch device tensors; methods marshal to the C ABI."""

    def __init__(self, shape, lo, hi, **kw):
        import torch
        self.torch = torch
        self.shape = tuple(int(n) for n in shape)
        self.N = int(np.prod(self.shape))
        self.precision = kw.get("precision", "fp64")
        self.dtype = torch.float32 if self.precision in ("fp32", "float32") else torch.float64
        self.batch = int(kw.get("batch", 1) or 1)
        self.max_batch = int(kw.get("max_batch", 1) or 1)
        self.model = kw.get("model", "seismic")
        desc, keep = make_desc(shape, lo, hi, **kw)
        self.handle = vofl_plan(desc, self._stream())
        self._keep = keep

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def _check_tensor(self, x, nfields, name):
        t = self.torch
        if not isinstance(x, t.Tensor) or not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if x.dtype != self.dtype:
            raise TypeError(f"{name} must have dtype {self.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if x.numel() != nfields * self.N:
            raise ValueError(f"{name} must hold {nfields} x {self.N} values")

    def apply(self, op: int, u, out=None):
        nf = u.numel() // self.N
        self._check_tensor(u, nf, "u")
        if out is None:
            out = self.torch.empty_like(u)
        self._check_tensor(out, nf, "out")
        vofl_apply(self.handle, op, u.data_ptr(), out.data_ptr(), nf, self._stream())
        return out

    def step(self, u, v, nsteps: int):
        self._check_tensor(u, self.batch, "u")
        self._check_tensor(v, self.batch, "v")
        vofl_step(self.handle, u.data_ptr(), v.data_ptr(), int(nsteps), self._stream())
        return u, v

    def step_graph(self, u, v, nsteps: int):
        self._check_tensor(u, self.batch, "u")
        self._check_tensor(v, self.batch, "v")
        vofl_step_graph(self.handle, u.data_ptr(), v.data_ptr(), int(nsteps), self._stream())
        return u, v

    def begin(self, u, v):
        """vofl_step_begin: start a resumable run from (u, v) (read only)."""
        self._check_tensor(u, self.batch, "u")
        self._check_tensor(v, self.batch, "v")
        vofl_step_begin(self.handle, u.data_ptr(), v.data_ptr(), self._stream())

    def advance(self, nsteps: int, graph: bool = False):
        """vofl_step_advance: nsteps steps of the run (graph: replay a captured graph)."""
        vofl_step_advance(self.handle, int(nsteps), 1 if graph else 0, self._stream())

    def end(self, u, v):
        """vofl_step_end: write the run's current (u, v) into the given tensors."""
        self._check_tensor(u, self.batch, "u")
        self._check_tensor(v, self.batch, "v")
        vofl_step_end(self.handle, u.data_ptr(), v.data_ptr(), self._stream())
        return u, v

    def lffp_start(self, phi, psi):
        """Leap-frog start (3.4b, c): returns new tensors (u^0, u^1)."""
        self._check_tensor(phi, self.batch, "phi")
        self._check_tensor(psi, self.batch, "psi")
        u_prev = self.torch.empty_like(phi)
        u = self.torch.empty_like(phi)
        vofl_lffp_start(self.handle, phi.data_ptr(), psi.data_ptr(), u_prev.data_ptr(), u.data_ptr(),
                        self._stream())
        return u_prev, u

    def lffp_step(self, u_prev, u, nsteps: int):
        self._check_tensor(u_prev, self.batch, "u_prev")
        self._check_tensor(u, self.batch, "u")
        vofl_lffp_step(self.handle, u_prev.data_ptr(), u.data_ptr(), int(nsteps), self._stream())
        return u_prev, u

    def cnfp_step(self, u_prev, u, nsteps: int, tol: float = 1e-13, max_iter: int = 200) -> int:
        """Crank-Nicolson steps (3.2) in place; returns the BiCGSTAB iterations."""
        self._check_tensor(u_prev, self.batch, "u_prev")
        self._check_tensor(u, self.batch, "u")
        return vofl_cnfp_step(self.handle, u_prev.data_ptr(), u.data_ptr(), int(nsteps), tol, max_iter,
                              self._stream())

    def solve(self, u0, v0, nsteps: int, u=None, v=None):
        """vofl_solve: (u, v) = (u0, v0) advanced by nsteps; new tensors unless given
        (u0 and v0 may be the outputs themselves)."""
        self._check_tensor(u0, self.batch, "u0")
        self._check_tensor(v0, self.batch, "v0")
        u = self.torch.empty_like(u0) if u is None else u
        v = self.torch.empty_like(v0) if v is None else v
        self._check_tensor(u, self.batch, "u")
        self._check_tensor(v, self.batch, "v")
        vofl_solve(self.handle, u0.data_ptr(), v0.data_ptr(), int(nsteps), u.data_ptr(), v.data_ptr(),
                   self._stream())
        return u, v

    def sync_status(self) -> int:
        return vofl_sync_status(self.handle, self._stream())

    def set_timing(self, enable=True):
        vofl_set_timing(self.handle, enable)

    def kernel_times(self):
        return vofl_kernel_times(self.handle)

    def info(self):
        return vofl_plan_info(self.handle)

    def close(self):
        if self.handle:
            vofl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
