"""ctypes binding of libhotrg.so (include/hotrg.h).  Argument marshalling
only: every step of the coarse-graining runs in the HIP library.  If the
library is not built the first call raises; there is no fallback."""

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_size_t, c_void_p

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhotrg.so")

HOTRG_OK, HOTRG_ERR_INVALID, HOTRG_ERR_OOM, HOTRG_ERR_DEVICE, HOTRG_ERR_NUMERIC, \
    HOTRG_ERR_NOT_READY, HOTRG_ERR_CANCELLED = range(7)
HOTRG_ISING, HOTRG_XY, HOTRG_POTTS, HOTRG_RAW = range(4)
HOTRG_FP64, HOTRG_FP32, HOTRG_BF16X3 = range(3)
HOTRG_TRUNC_PLAIN, HOTRG_TRUNC_MULTIPLET = range(2)

PREC = {"fp64": HOTRG_FP64, "fp32": HOTRG_FP32, "bf16x3": HOTRG_BF16X3}
TRUNC = {"plain": HOTRG_TRUNC_PLAIN, "multiplet": HOTRG_TRUNC_MULTIPLET}
MODEL = {"ising": HOTRG_ISING, "xy": HOTRG_XY, "potts": HOTRG_POTTS, "raw": HOTRG_RAW}

EXPORTS = [
    "hotrg_ctx_create", "hotrg_ctx_destroy", "hotrg_last_error", "hotrg_ctx_bytes_in_use",
    "hotrg_init_tensor", "hotrg_step", "hotrg_finish", "hotrg_state_export", "hotrg_state_free",
    "hotrg_run", "hotrg_environment", "hotrg_coarse", "hotrg_ctx_enable_timing", "hotrg_ctx_timings",
]

PHASES = ["env", "eigh", "proj", "c1", "c2", "c3", "norm"]


class HotrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hotrg status %d: %s" % (status, msg))
        self.status = status


class ModelParams(ctypes.Structure):
    _fields_ = [("model", c_int), ("beta", c_double), ("J", c_double), ("n_max", c_int),
                ("q", c_int), ("raw", POINTER(c_double)), ("raw_dx", c_int), ("raw_dy", c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("d_cut", c_int), ("n_steps", c_int), ("prec", c_int), ("trunc", c_int),
                ("degen_tol", c_double), ("spec_len", c_int), ("eig", c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("dx", c_int), ("dy", c_int), ("d_new", c_int), ("kept", c_int),
                ("log_norm", c_double), ("trunc_err", c_double), ("cut_gap", c_double),
                ("lnz_torus", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PhaseTime(ctypes.Structure):
    _fields_ = [("step", c_int), ("phase", c_int), ("dx", c_int), ("dy", c_int),
                ("d_new", c_int), ("ms", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("lnz_per_site", c_double), ("n_steps", c_int), ("steps", POINTER(StepInfo)),
                ("spectra", POINTER(c_double)), ("seconds", c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhotrg.so is not built: run `python -m paper_2306_00358_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    L.hotrg_last_error.restype = ctypes.c_char_p
    L.hotrg_ctx_create.argtypes = [c_int, vp, c_size_t, POINTER(vp)]
    L.hotrg_ctx_destroy.argtypes = [vp]
    L.hotrg_ctx_destroy.restype = None
    L.hotrg_ctx_bytes_in_use.argtypes = [vp]
    L.hotrg_ctx_bytes_in_use.restype = c_size_t
    L.hotrg_init_tensor.argtypes = [vp, POINTER(ModelParams), c_int, POINTER(vp)]
    L.hotrg_step.argtypes = [vp, vp, POINTER(Opts), POINTER(StepInfo), POINTER(c_double)]
    L.hotrg_finish.argtypes = [vp, vp, POINTER(c_double)]
    L.hotrg_state_export.argtypes = [vp, vp, POINTER(c_double), c_size_t, POINTER(c_int),
                                     POINTER(c_double), POINTER(c_int)]
    L.hotrg_state_free.argtypes = [vp, vp]
    L.hotrg_state_free.restype = None
    L.hotrg_run.argtypes = [vp, POINTER(ModelParams), POINTER(Opts), POINTER(Result)]
    L.hotrg_environment.argtypes = [vp, c_int, vp, c_int, c_int, vp]
    L.hotrg_coarse.argtypes = [vp, c_int, vp, vp, c_int, c_int, c_int, vp, vp]
    L.hotrg_ctx_enable_timing.argtypes = [vp, c_int]
    L.hotrg_ctx_timings.argtypes = [vp, POINTER(PhaseTime), c_int]
    for name in EXPORTS:
        if name not in ("hotrg_ctx_destroy", "hotrg_state_free", "hotrg_last_error",
                        "hotrg_ctx_bytes_in_use"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def _check(status):
    if status != HOTRG_OK:
        raise HotrgError(status, lib().hotrg_last_error().decode())


def model_params(model="ising", beta=0.44, J=1.0, n_max=0, q=2, raw=None):
    """ModelParams for a named model; `raw` is an array (dx, dy, dx, dy)."""
    p = ModelParams()
    p.model = MODEL[model] if isinstance(model, str) else int(model)
    p.beta, p.J, p.n_max, p.q = float(beta), float(J), int(n_max), int(q)
    p._keep = None
    if raw is not None:
        a = np.ascontiguousarray(raw, dtype=np.float64)
        if a.ndim != 4:
            raise ValueError("raw tensor must be rank 4")
        p.raw = a.ctypes.data_as(POINTER(c_double))
        p.raw_dx, p.raw_dy = a.shape[0], a.shape[1]
        p._keep = a
    return p


EIG = {"auto": 0, "dense": 1}


def make_opts(d_cut, n_steps=0, prec="fp64", trunc="plain", degen_tol=1e-10, spec_len=0,
              eig="auto"):
    o = Opts()
    o.eig = EIG[eig] if isinstance(eig, str) else int(eig)
    o.d_cut, o.n_steps = int(d_cut), int(n_steps)
    o.prec = PREC[prec] if isinstance(prec, str) else int(prec)
    o.trunc = TRUNC[trunc] if isinstance(trunc, str) else int(trunc)
    o.degen_tol, o.spec_len = float(degen_tol), int(spec_len)
    return o


class Context:
    """hotrg_ctx on one GPU.  `stream` is a raw hipStream_t handle (int) or
    None for the library's own stream."""

    def __init__(self, device=0, stream=None, hbm_budget=0):
        self.ptr = c_void_p()
        _check(lib().hotrg_ctx_create(int(device), c_void_p(stream) if stream else None,
                                      int(hbm_budget), byref(self.ptr)))

    def close(self):
        if self.ptr:
            lib().hotrg_ctx_destroy(self.ptr)
            self.ptr = c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bytes_in_use(self):
        return lib().hotrg_ctx_bytes_in_use(self.ptr)

    def enable_timing(self, on=True):
        _check(lib().hotrg_ctx_enable_timing(self.ptr, 1 if on else 0))

    def timings(self, cap=1 << 16):
        """Per-phase records since the last call: list of dicts with keys
        step, phase (name), dx, dy, d_new, ms."""
        buf = (PhaseTime * cap)()
        n = lib().hotrg_ctx_timings(self.ptr, buf, cap)
        if n < 0:
            raise HotrgError(HOTRG_ERR_DEVICE, lib().hotrg_last_error().decode())
        return [{"step": b.step, "phase": PHASES[b.phase], "dx": b.dx, "dy": b.dy,
                 "d_new": b.d_new, "ms": b.ms} for b in buf[:n]]


def hotrg_run(ctx, params, opts):
    """Whole run.  Returns dict(lnz_per_site, steps=[dict], spectra=(n_steps, spec_len), seconds)."""
    K = opts.n_steps
    infos = (StepInfo * max(K, 1))()
    spec = np.zeros((max(K, 1), max(opts.spec_len, 1)), dtype=np.float64)
    r = Result()
    r.steps = ctypes.cast(infos, POINTER(StepInfo))
    r.spectra = spec.ctypes.data_as(POINTER(c_double)) if opts.spec_len else None
    _check(lib().hotrg_run(ctx.ptr, byref(params), byref(opts), byref(r)))
    return {"lnz_per_site": r.lnz_per_site, "n_steps": r.n_steps,
            "steps": [infos[i].as_dict() for i in range(K)],
            "spectra": spec[:K, :opts.spec_len], "seconds": r.seconds}


class State:
    """A coarse-graining state (hotrg_init_tensor ... hotrg_state_free)."""

    def __init__(self, ctx, params, prec="fp64"):
        self.ctx = ctx
        self.ptr = c_void_p()
        p = PREC[prec] if isinstance(prec, str) else int(prec)
        _check(lib().hotrg_init_tensor(ctx.ptr, byref(params), p, byref(self.ptr)))

    def step(self, opts, want_info=True):
        info = StepInfo()
        spec = np.zeros(max(opts.spec_len, 1))
        if want_info:
            _check(lib().hotrg_step(self.ctx.ptr, self.ptr, byref(opts), byref(info),
                                    spec.ctypes.data_as(POINTER(c_double)) if opts.spec_len else None))
            return info.as_dict(), spec[:opts.spec_len]
        _check(lib().hotrg_step(self.ctx.ptr, self.ptr, byref(opts), None, None))
        return None, None

    def finish(self):
        v = c_double()
        _check(lib().hotrg_finish(self.ctx.ptr, self.ptr, byref(v)))
        return v.value

    def export(self):
        dims = (c_int * 2)()
        acc, k = c_double(), c_int()
        _check(lib().hotrg_state_export(self.ctx.ptr, self.ptr, None, 0, dims, byref(acc), byref(k)))
        dx, dy = dims[0], dims[1]
        buf = np.zeros((dx, dy, dx, dy), dtype=np.float64)
        _check(lib().hotrg_state_export(self.ctx.ptr, self.ptr, buf.ctypes.data_as(POINTER(c_double)),
                                        buf.size, dims, byref(acc), byref(k)))
        return buf, acc.value, k.value

    def free(self):
        if self.ptr:
            lib().hotrg_state_free(self.ctx.ptr, self.ptr)
            self.ptr = c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def hotrg_environment(ctx, T, M, prec="fp64"):
    """Environment on device buffers: T (dx,dy,dx,dy) float64 tensor -> M (dx^2, dx^2)."""
    dx, dy = T.shape[0], T.shape[1]
    _check(lib().hotrg_environment(ctx.ptr, _prec(prec), c_void_p(T.data_ptr()), dx, dy,
                                   c_void_p(M.data_ptr())))


def hotrg_coarse(ctx, T, U, Tt, max_abs=None, prec="fp64"):
    """Coarse tensor on device buffers: T (dx,dy,dx,dy), U (dx,dx,dn) -> Tt (dn,dy,dn,dy)."""
    dx, dy, dn = T.shape[0], T.shape[1], U.shape[2]
    _check(lib().hotrg_coarse(ctx.ptr, _prec(prec), c_void_p(T.data_ptr()), c_void_p(U.data_ptr()),
                              dx, dy, dn, c_void_p(Tt.data_ptr()),
                              c_void_p(max_abs.data_ptr()) if max_abs is not None else None))
