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
HOTRG_ISING, HOTRG_XY, HOTRG_POTTS, HOTRG_RAW, HOTRG_GXY = range(5)
HOTRG_FP64, HOTRG_FP32, HOTRG_BF16X3, HOTRG_PREC_AUTO = range(4)
HOTRG_TRUNC_PLAIN, HOTRG_TRUNC_MULTIPLET = range(2)
HOTRG_ISO_ONE_SIDED, HOTRG_ISO_TWO_SIDED = range(2)

PREC = {"fp64": HOTRG_FP64, "fp32": HOTRG_FP32, "bf16x3": HOTRG_BF16X3, "auto": HOTRG_PREC_AUTO}
TRUNC = {"plain": HOTRG_TRUNC_PLAIN, "multiplet": HOTRG_TRUNC_MULTIPLET}
MODEL = {"ising": HOTRG_ISING, "xy": HOTRG_XY, "potts": HOTRG_POTTS, "raw": HOTRG_RAW,
         "gxy": HOTRG_GXY}
ISOMETRY = {"one": HOTRG_ISO_ONE_SIDED, "two": HOTRG_ISO_TWO_SIDED}

EXPORTS = [
    "hotrg_ctx_create", "hotrg_ctx_destroy", "hotrg_last_error", "hotrg_ctx_bytes_in_use",
    "hotrg_init_tensor", "hotrg_step", "hotrg_finish", "hotrg_state_export", "hotrg_state_free",
    "hotrg_run", "hotrg_environment", "hotrg_coarse", "hotrg_ctx_enable_timing", "hotrg_ctx_timings",
    "hotrg_ctx_set_workers", "hotrg_submit", "hotrg_poll", "hotrg_wait", "hotrg_cancel",
    "hotrg_footprint", "hotrg_run_batch", "hotrg_ctx_sched_stats", "hotrg_thermo",
    "hotrg_release", "hotrg_coarse_noalloc", "hotrg_plan", "hotrg_run_grouped",
    "hotrg_ctx_group_stats", "hotrg_projector", "hotrg_ctx_last_eig",
]

NOALLOC_SCRATCH_BYTES = 64 << 20  # HOTRG_NOALLOC_SCRATCH_BYTES

PHASES = ["env", "eigh", "proj", "c1", "c2", "c3", "norm"]


class HotrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hotrg status %d: %s" % (status, msg))
        self.status = status


class ModelParams(ctypes.Structure):
    _fields_ = [("model", c_int), ("beta", c_double), ("J", c_double), ("n_max", c_int),
                ("q", c_int), ("raw", POINTER(c_double)), ("raw_dx", c_int), ("raw_dy", c_int),
                ("delta", c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("d_cut", c_int), ("n_steps", c_int), ("prec", c_int), ("trunc", c_int),
                ("degen_tol", c_double), ("spec_len", c_int), ("eig", c_int),
                ("isometry", c_int), ("tol", c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("dx", c_int), ("dy", c_int), ("d_new", c_int), ("kept", c_int),
                ("log_norm", c_double), ("trunc_err", c_double), ("cut_gap", c_double),
                ("lnz_torus", c_double), ("side", c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PhaseTime(ctypes.Structure):
    _fields_ = [("step", c_int), ("phase", c_int), ("dx", c_int), ("dy", c_int),
                ("d_new", c_int), ("ms", ctypes.c_float)]


class Result(ctypes.Structure):
    _fields_ = [("lnz_per_site", c_double), ("n_steps", c_int), ("steps", POINTER(StepInfo)),
                ("spectra", POINTER(c_double)), ("seconds", c_double), ("t_submit", c_double),
                ("t_start", c_double), ("t_end", c_double), ("prec_used", c_int),
                ("err_bound", c_double)]


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
    L.hotrg_coarse_noalloc.argtypes = [vp, vp, vp, c_int, c_int, c_int, vp, vp]
    L.hotrg_projector.argtypes = [vp, vp, c_int, c_int, c_int, c_double, c_int, vp,
                                  POINTER(c_double), POINTER(c_int), POINTER(c_double)]
    L.hotrg_ctx_enable_timing.argtypes = [vp, c_int]
    L.hotrg_ctx_last_eig.argtypes = [vp, POINTER(c_int), POINTER(c_double)]
    L.hotrg_ctx_set_workers.argtypes = [vp, c_int]
    L.hotrg_submit.argtypes = [vp, POINTER(ModelParams), POINTER(Opts), POINTER(Result),
                               POINTER(ctypes.c_uint64)]
    L.hotrg_poll.argtypes = [vp, ctypes.c_uint64]
    L.hotrg_wait.argtypes = [vp, ctypes.c_uint64, c_double]
    L.hotrg_cancel.argtypes = [vp, ctypes.c_uint64]
    L.hotrg_release.argtypes = [vp, ctypes.c_uint64]
    L.hotrg_footprint.argtypes = [POINTER(ModelParams), POINTER(Opts), POINTER(c_size_t)]
    L.hotrg_plan.argtypes = [POINTER(ModelParams), POINTER(Opts), POINTER(c_int), POINTER(c_int),
                             POINTER(c_double)]
    L.hotrg_run_batch.argtypes = [vp, c_int, POINTER(ModelParams), POINTER(Opts), POINTER(Result),
                                  POINTER(c_int)]
    L.hotrg_run_grouped.argtypes = [vp, c_int, POINTER(ModelParams), POINTER(Opts),
                                    POINTER(Result), POINTER(c_int)]
    L.hotrg_ctx_group_stats.argtypes = [vp] + [POINTER(ctypes.c_uint64)] * 4
    L.hotrg_ctx_sched_stats.argtypes = [vp, POINTER(ctypes.c_uint64), POINTER(ctypes.c_uint64),
                                        POINTER(c_size_t)]
    L.hotrg_ctx_timings.argtypes = [vp, POINTER(PhaseTime), c_int]
    L.hotrg_thermo.argtypes = [vp, POINTER(ModelParams), POINTER(Opts), c_double, POINTER(c_double)]
    for name in EXPORTS:
        if name not in ("hotrg_ctx_destroy", "hotrg_state_free", "hotrg_last_error",
                        "hotrg_ctx_bytes_in_use"):
            getattr(L, name).restype = c_int
    _lib = L
    return L


def _check(status):
    if status != HOTRG_OK:
        raise HotrgError(status, lib().hotrg_last_error().decode())


def model_params(model="ising", beta=0.44, J=1.0, n_max=0, q=2, raw=None, delta=1.0):
    """ModelParams for a named model; `raw` is an array (dx, dy, dx, dy)."""
    p = ModelParams()
    p.model = MODEL[model] if isinstance(model, str) else int(model)
    p.beta, p.J, p.n_max, p.q = float(beta), float(J), int(n_max), int(q)
    p.delta = float(delta)
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
              eig="auto", isometry="one", tol=0.0):
    o = Opts()
    o.tol = float(tol)
    o.eig = EIG[eig] if isinstance(eig, str) else int(eig)
    o.isometry = ISOMETRY[isometry] if isinstance(isometry, str) else int(isometry)
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

    def set_workers(self, n):
        _check(lib().hotrg_ctx_set_workers(self.ptr, int(n)))

    def sched_stats(self):
        a, st, pk = ctypes.c_uint64(), ctypes.c_uint64(), c_size_t()
        _check(lib().hotrg_ctx_sched_stats(self.ptr, byref(a), byref(st), byref(pk)))
        return {"admitted": a.value, "stalls": st.value, "peak_reserved": pk.value}

    def group_stats(self):
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().hotrg_ctx_group_stats(self.ptr, *[byref(x) for x in v]))
        return dict(zip(("sweeps", "replays", "captures", "fallbacks"), (x.value for x in v)))

    def enable_timing(self, on=True):
        _check(lib().hotrg_ctx_enable_timing(self.ptr, 1 if on else 0))

    def last_eig(self):
        """(sweeps, resid) of the context's last leading-eigenpair solve;
        sweeps = 0 for a dense one."""
        sw, rs = c_int(0), c_double(0.0)
        _check(lib().hotrg_ctx_last_eig(self.ptr, byref(sw), byref(rs)))
        return sw.value, rs.value

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
            "spectra": spec[:K, :opts.spec_len], "seconds": r.seconds, "prec_used": r.prec_used,
            "err_bound": r.err_bound}


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


def hotrg_projector(ctx, M, U, d_new, trunc="plain", degen_tol=1e-10, spec_len=0):
    """Projector on device buffers: M (n, n) float64 environment -> U (n, d_new)
    float64, the eigenvectors of the d_new largest eigenvalues (columns past
    the kept count zero).  Returns (kept, truncation error, spectrum list)."""
    n = M.shape[0]
    spec = (c_double * max(spec_len, 1))()
    kept = c_int(0)
    err = c_double(0.0)
    _check(lib().hotrg_projector(ctx.ptr, c_void_p(M.data_ptr()), n, d_new, TRUNC[trunc],
                                 degen_tol, spec_len, c_void_p(U.data_ptr()),
                                 spec if spec_len else None, ctypes.byref(kept),
                                 ctypes.byref(err)))
    return kept.value, err.value, list(spec[:spec_len])


def hotrg_coarse_noalloc(ctx, T, U, Tt, max_abs=None):
    """hotrg_coarse in FP64 without any allocation (intermediates in the
    library's static scratch array); enqueued on the context's stream, not
    waited for: synchronise before reading Tt."""
    dx, dy, dn = T.shape[0], T.shape[1], U.shape[2]
    _check(lib().hotrg_coarse_noalloc(ctx.ptr, c_void_p(T.data_ptr()), c_void_p(U.data_ptr()),
                                      dx, dy, dn, c_void_p(Tt.data_ptr()),
                                      c_void_p(max_abs.data_ptr()) if max_abs is not None else None))


def _result_dict(r, infos, spec, K, spec_len):
    return {"lnz_per_site": r.lnz_per_site, "n_steps": r.n_steps,
            "steps": [infos[i].as_dict() for i in range(K)] if infos is not None else [],
            "spectra": spec[:K, :spec_len] if spec is not None else None,
            "seconds": r.seconds, "t_submit": r.t_submit, "t_start": r.t_start, "t_end": r.t_end,
            "prec_used": r.prec_used, "err_bound": r.err_bound}


def hotrg_plan(params, opts):
    """The precision schedule of a run: dict(prec, first_reduced, err_bound)."""
    p, k0, e = c_int(), c_int(), c_double()
    _check(lib().hotrg_plan(byref(params), byref(opts), byref(p), byref(k0), byref(e)))
    return {"prec": p.value, "first_reduced": k0.value, "err_bound": e.value}


def hotrg_footprint(params, opts):
    b = c_size_t()
    _check(lib().hotrg_footprint(byref(params), byref(opts), byref(b)))
    return b.value


def hotrg_run_grouped(ctx, params_list, opts_list, with_steps=False):
    """Run problems in lockstep (grouped launches, one graph per sweep);
    returns (list of result dicts or None for failed problems, statuses)."""
    return hotrg_run_batch(ctx, params_list, opts_list, with_steps, _fn="hotrg_run_grouped")


def hotrg_run_batch(ctx, params_list, opts_list, with_steps=False, _fn="hotrg_run_batch"):
    """Run problems on the context's worker pool; returns (list of result
    dicts or None for failed problems, list of statuses)."""
    n = len(params_list)
    P = (ModelParams * n)(*params_list)
    O = (Opts * n)(*opts_list)
    R = (Result * n)()
    keep = []
    for i, o in enumerate(opts_list):
        if with_steps:
            infos = (StepInfo * max(o.n_steps, 1))()
            spec = np.zeros((max(o.n_steps, 1), max(o.spec_len, 1)))
            R[i].steps = ctypes.cast(infos, POINTER(StepInfo))
            R[i].spectra = spec.ctypes.data_as(POINTER(c_double)) if o.spec_len else None
            keep.append((infos, spec))
        else:
            keep.append((None, None))
    S = (c_int * n)()
    getattr(lib(), _fn)(ctx.ptr, n, P, O, R, S)
    out = []
    for i in range(n):
        if S[i] != HOTRG_OK:
            out.append(None)
        else:
            infos, spec = keep[i]
            out.append(_result_dict(R[i], infos, spec, opts_list[i].n_steps, opts_list[i].spec_len))
    return out, [int(x) for x in S]


class Ticket:
    """A submitted problem: the result buffers live here until it completes."""

    def __init__(self, ctx, params, opts, with_steps=False):
        self.ctx, self.params, self.opts = ctx, params, opts
        self.result = Result()
        self.infos = self.spec = None
        if with_steps:
            self.infos = (StepInfo * max(opts.n_steps, 1))()
            self.spec = np.zeros((max(opts.n_steps, 1), max(opts.spec_len, 1)))
            self.result.steps = ctypes.cast(self.infos, POINTER(StepInfo))
            self.result.spectra = (self.spec.ctypes.data_as(POINTER(c_double))
                                   if opts.spec_len else None)
        self.id = ctypes.c_uint64()
        _check(lib().hotrg_submit(ctx.ptr, byref(params), byref(opts), byref(self.result),
                                  byref(self.id)))

    def poll(self):
        return lib().hotrg_poll(self.ctx.ptr, self.id)

    def wait(self, timeout=-1.0):
        return lib().hotrg_wait(self.ctx.ptr, self.id, float(timeout))

    def cancel(self):
        _check(lib().hotrg_cancel(self.ctx.ptr, self.id))

    def release(self):
        """Forget the finished ticket (hotrg_release)."""
        _check(lib().hotrg_release(self.ctx.ptr, self.id))

    def value(self):
        """Wait, release the ticket and return the result (raises on failure)."""
        st = self.wait()
        err = lib().hotrg_last_error().decode() if st != HOTRG_OK else ""
        if st != HOTRG_ERR_NOT_READY:
            self.release()
        if st != HOTRG_OK:
            raise HotrgError(st, err)
        return _result_dict(self.result, self.infos, self.spec, self.opts.n_steps, self.opts.spec_len)


def hotrg_thermo(ctx, params, opts, dbeta):
    """ln Z/N, energy per site and specific heat per site at params.beta by
    five-point differences over beta +- dbeta, +- 2 dbeta (hotrg_thermo)."""
    out = (c_double * 3)()
    _check(lib().hotrg_thermo(ctx.ptr, byref(params), byref(opts), float(dbeta), out))
    return {"lnz": out[0], "energy": out[1], "cv": out[2]}
