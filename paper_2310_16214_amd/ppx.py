"""ctypes binding of libppx.so (declared in include/ppx.h).

Argument marshalling only: every operation runs in the library's HIP
kernels.  Buffers may be passed as torch tensors (their ``data_ptr()`` is
used) or as raw integer device addresses.  When ``stream`` is None and a
torch tensor is given, torch's current HIP stream is used so that the call is
ordered with the caller's torch work.  A missing library raises at first use.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libppx.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "ppx.h")
HEADERS = [HEADER] + [os.path.join(os.path.dirname(_PKG), "include", h)
                      for h in ("ppx_tune.h", "ppx_serve.h")]

# ---- constants mirrored from include/ppx.h ----
OK, EINVAL, ECONFIG, EDEVICE, EHIP, ENOMEM, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
I32, F32, F64, C64 = 0, 1, 2, 3
OP_FFT, OP_SCAN, OP_TRIDIAG = 0, 1, 2
FFT_LDS, FFT_LDS_SPLIT, FFT_LDS_PIPE, FFT_LDS_SPLIT_PIPE = 0, 1, 2, 3
SCAN_KS, SCAN_LF, SCAN_KS_PIPE, SCAN_LF_PIPE = 0, 1, 2, 3
TRI_CR, TRI_PCR, TRI_CR_PCR, TRI_CR_SHFL, TRI_PCR_SHFL, TRI_PCR_REG, TRI_WM, TRI_LF = 0, 1, 2, 3, 4, 5, 6, 7
TRI_PIPE = 8  # flag on an in-wave variant: persistent workgroups with prefetch


def tri_family(algo):
    """TRI_CR for the CR variants, TRI_PCR for the PCR variants; the CR -> PCR
    hybrid, Wang & Mou and Ladner-Fischer are families of their own."""
    base = algo & ~TRI_PIPE
    return (TRI_CR if base in (TRI_CR, TRI_CR_SHFL) else TRI_PCR if base in (TRI_PCR, TRI_PCR_SHFL, TRI_PCR_REG)
            else base)
TUNE_EXHAUSTIVE, TUNE_ANALYTICAL, TUNE_LEARNED = 0, 1, 2
MIN_N, MAX_N = 16, 16384


class PpxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ppx error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    """ppx_config: (radix r, P, L, G_b, S, algo)."""
    _fields_ = [("radix", ctypes.c_int32),
                ("elems_per_thread", ctypes.c_int32),
                ("threads_per_block", ctypes.c_int32),
                ("problems_per_block", ctypes.c_int32),
                ("lds_elems", ctypes.c_int32),
                ("algo", ctypes.c_int32)]

    def as_tuple(self):
        return (self.radix, self.elems_per_thread, self.threads_per_block,
                self.problems_per_block, self.lds_elems, self.algo)

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "Config(r=%d, P=%d, L=%d, G_b=%d, S=%d, algo=%d)" % self.as_tuple()


def make_config(radix=2, threads_per_block=64, problems_per_block=1, algo=0,
                elems_per_thread=0, lds_elems=0) -> Config:
    return Config(radix, elems_per_thread, threads_per_block, problems_per_block,
                  lds_elems, algo)


_lib = None
_lock = threading.Lock()


def header_functions(paths=None):
    """Names of the functions declared in the include/*.h headers."""
    names = []
    for path in paths or HEADERS:
        txt = open(path).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"typedef[^;]*;", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return names


def lib():
    """Load libppx.so (raises if it has not been built).

    torch bundles its own HIP runtime under the same soname as ROCm's
    (libamdhip64.so.7).  Importing torch first makes the dynamic linker bind
    libppx.so to that already-loaded runtime, so the process holds a single
    HIP runtime and torch's device pointers and streams are valid here.
    """
    global _lib
    with _lock:
        if _lib is None:
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2310_16214_amd.build` (no CPU fallback exists)")
            L = ctypes.CDLL(LIB_PATH)
            vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
            cfgp = ctypes.POINTER(Config)
            L.fft_batched.argtypes = [vp, vp, i64, i64, ci, cfgp, vp]
            L.scan_batched.argtypes = [vp, vp, i64, i64, ci, cfgp, vp]
            L.scan_exclusive_batched.argtypes = [vp, vp, i64, i64, ci, cfgp, vp]
            L.tridiag_batched.argtypes = [vp, vp, vp, vp, vp, i64, i64, ci, cfgp, vp]
            L.tune.argtypes = [ci, ci, i64, i64, ci, ci, cfgp,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ci)]
            L.ppx_last_error.restype = ctypes.c_char_p
            L.ppx_last_error.argtypes = []
            L.ppx_config_valid.argtypes = [ci, ci, i64, cfgp]
            L.ppx_default_config.argtypes = [ci, ci, i64, cfgp]
            L.ppx_resolve_config.argtypes = [ci, ci, i64, i64, cfgp]
            L.ppx_enumerate_configs.argtypes = [ci, ci, i64, cfgp, ci]
            for name in ("fft_batched", "scan_batched", "scan_exclusive_batched",
                         "tridiag_batched", "tune",
                         "ppx_config_valid", "ppx_default_config", "ppx_resolve_config",
                         "ppx_enumerate_configs"):
                getattr(L, name).restype = ci
            _lib = L
    return _lib


def last_error() -> str:
    return lib().ppx_last_error().decode()


def _check(rc):
    if rc < 0:
        raise PpxError(rc, last_error())
    return rc


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return int(x)


def _stream(stream, *tensors):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    for t in tensors:
        if hasattr(t, "is_cuda") and t.is_cuda:
            import torch
            return torch.cuda.current_stream(t.device).cuda_stream
    return None


def _cfgp(cfg):
    return ctypes.byref(cfg) if cfg is not None else None


def fft_batched(inp, out, n, batch, direction=-1, cfg=None, stream=None):
    """Batched complex FFT (see include/ppx.h)."""
    _check(lib().fft_batched(_ptr(inp), _ptr(out), n, batch, direction, _cfgp(cfg),
                             _stream(stream, inp, out)))


def scan_batched(inp, out, n, batch, dtype, cfg=None, stream=None):
    """Batched inclusive sum scan, dtype I32, F32 or F64."""
    _check(lib().scan_batched(_ptr(inp), _ptr(out), n, batch, dtype, _cfgp(cfg),
                              _stream(stream, inp, out)))


def scan_exclusive_batched(inp, out, n, batch, dtype, cfg=None, stream=None):
    """Batched exclusive sum scan (out[0] = 0), dtype I32, F32 or F64."""
    _check(lib().scan_exclusive_batched(_ptr(inp), _ptr(out), n, batch, dtype, _cfgp(cfg),
                                        _stream(stream, inp, out)))


def tridiag_batched(a, b, c, d, x, n, batch, dtype, cfg=None, stream=None):
    """Batched tridiagonal solve, dtype F32 or F64."""
    _check(lib().tridiag_batched(_ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), n, batch,
                                 dtype, _cfgp(cfg), _stream(stream, a, b, c, d, x)))


def tune(op, dtype, n, batch, method, max_evals=0):
    """Returns (Config, best_us, evals_used)."""
    best = Config()
    us = ctypes.c_double(0.0)
    ev = ctypes.c_int(0)
    _check(lib().tune(op, dtype, n, batch, method, max_evals, ctypes.byref(best),
                      ctypes.byref(us), ctypes.byref(ev)))
    return best, us.value, ev.value


def config_valid(op, dtype, n, cfg) -> bool:
    return lib().ppx_config_valid(op, dtype, n, ctypes.byref(cfg)) == OK


def default_config(op, dtype, n) -> Config:
    c = Config()
    _check(lib().ppx_default_config(op, dtype, n, ctypes.byref(c)))
    return c


def resolve_config(op, dtype, n, batch) -> Config:
    c = Config()
    _check(lib().ppx_resolve_config(op, dtype, n, batch, ctypes.byref(c)))
    return c


def enumerate_configs(op, dtype, n):
    cnt = _check(lib().ppx_enumerate_configs(op, dtype, n, None, 0))
    arr = (Config * max(cnt, 1))()
    _check(lib().ppx_enumerate_configs(op, dtype, n, arr, cnt))
    return [arr[i] for i in range(cnt)]


# ---------------------------------------------------------------- tuning engine
# (declared in include/ppx_tune.h)

class DeviceModel(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in (
        "wave_size", "partitions", "regs_per_partition", "reg_granule", "max_waves_per_cu",
        "max_blocks_per_cu", "lds_per_cu", "lds_per_block", "lds_granule", "num_cus")]


class Resource(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("regs_per_thread", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("best", Config), ("best_us", ctypes.c_double), ("evals_used", ctypes.c_int32),
                ("ncands", ctypes.c_int32), ("trace_cfg", ctypes.POINTER(Config)),
                ("trace_us", ctypes.POINTER(ctypes.c_double)), ("trace_cap", ctypes.c_int32)]


EVAL_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(Config), ctypes.c_void_p)
ANALYTICAL_GRID_FILL, ANALYTICAL_WINDOW_50 = 1, 4

class FftPlan(ctypes.Structure):
    """ppx_fft_plan: (log2 n1, radix and tile width of pass A and of pass B)."""
    _fields_ = [("log2_n1", ctypes.c_int32), ("radix_a", ctypes.c_int32), ("radix_b", ctypes.c_int32),
                ("tile_a", ctypes.c_int32), ("tile_b", ctypes.c_int32)]

    def as_tuple(self):
        return (self.log2_n1, self.radix_a, self.radix_b, self.tile_a, self.tile_b)

    def __repr__(self):
        return "FftPlan(log2_n1=%d, radix_a=%d, radix_b=%d, tile_a=%d, tile_b=%d)" % self.as_tuple()


MAX_N = 16384
MAX_N_LARGE = 1 << 23

_tune_sigs = {
    "fft_batched_large": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                           ctypes.POINTER(FftPlan), ctypes.c_void_p], ctypes.c_int),
    "ppx_fft_plan_valid": ([ctypes.c_int64, ctypes.POINTER(FftPlan)], ctypes.c_int),
    "ppx_enumerate_fft_plans": ([ctypes.c_int64, ctypes.POINTER(FftPlan), ctypes.c_int], ctypes.c_int),
    "ppx_default_fft_plan": ([ctypes.c_int64, ctypes.POINTER(FftPlan)], ctypes.c_int),
    "tune_fft_large": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(FftPlan),
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ppx_tune_large_trace": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(FftPlan), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(FftPlan), ctypes.POINTER(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "ppx_occupancy": ([ctypes.POINTER(DeviceModel), ctypes.POINTER(Resource),
                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "ppx_device_model_gfx950": ([ctypes.POINTER(DeviceModel)], ctypes.c_int),
    "ppx_analytical_pick": ([ctypes.POINTER(DeviceModel), ctypes.POINTER(Config),
                             ctypes.POINTER(Resource), ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ppx_analytical_select": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(Config),
                               ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ppx_bo_search": ([ctypes.POINTER(Config), ctypes.c_int, EVAL_FN, ctypes.c_void_p, ctypes.c_int,
                       ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "ppx_gp_posterior": ([ctypes.POINTER(ctypes.c_double)] * 2 + [ctypes.c_int] * 2 +
                         [ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double,
                          ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                         ctypes.c_int),
    "ppx_expected_improvement": ([ctypes.c_double] * 3, ctypes.c_double),
    "ppx_tune_ex": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(TuneReport)],
                    ctypes.c_int),
    "ppx_time_config": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                         ctypes.POINTER(Config), ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
                        ctypes.c_int),
    "ppx_stream_reference": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                              ctypes.c_void_p], ctypes.c_int),
    "ppx_kernel_resources": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(Config),
                              ctypes.POINTER(Resource)], ctypes.c_int),
    "ppx_tune_cache_load": ([ctypes.c_char_p], ctypes.c_int),
    "ppx_tune_cache_save": ([ctypes.c_char_p], ctypes.c_int),
    "ppx_tune_cache_clear": ([], ctypes.c_int),
    "ppx_tuned_config": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                          ctypes.POINTER(Config)], ctypes.c_int),
}


_tune_sigs.update({
    "ppx_online_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                           ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "ppx_online_next": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Config)], ctypes.c_int),
    "ppx_online_report": ([ctypes.c_void_p, ctypes.c_double], ctypes.c_int),
    "ppx_online_status": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "ppx_online_destroy": ([ctypes.c_void_p], ctypes.c_int),
})


def _tl(name):
    f = getattr(lib(), name)
    if not getattr(f, "_ppx_typed", False):
        f.argtypes, f.restype = _tune_sigs[name]
        f._ppx_typed = True
    return f


class OnlineTuner:
    """Online learned-tuning session (ppx_online_* in include/ppx_tune.h)."""

    def __init__(self, op, dtype, n, batch, algo=-1, max_evals=0):
        self._h = ctypes.c_void_p()
        _check(_tl("ppx_online_create")(op, dtype, n, batch, algo, max_evals, ctypes.byref(self._h)))

    def next(self, explore=True):
        """(config, is_candidate): is_candidate means report() its cost next."""
        c = Config()
        r = _check(_tl("ppx_online_next")(self._h, 1 if explore else 0, ctypes.byref(c)))
        return c, r == 1

    def report(self, cost):
        _check(_tl("ppx_online_report")(self._h, float(cost)))

    def status(self):
        ev, conv, best, cost = ctypes.c_int(0), ctypes.c_int(0), Config(), ctypes.c_double(0)
        _check(_tl("ppx_online_status")(self._h, ctypes.byref(ev), ctypes.byref(conv), ctypes.byref(best),
                                         ctypes.byref(cost)))
        return dict(evals=ev.value, converged=bool(conv.value), best=best, best_cost=cost.value)

    def close(self):
        if self._h:
            _tl("ppx_online_destroy")(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fft_batched_large(inp, out, n, batch, direction=-1, plan=None, stream=None):
    """Two-pass FFT for 16384 < n <= 2^23 (see include/ppx.h); in and out must
    not overlap."""
    _check(_tl("fft_batched_large")(_ptr(inp), _ptr(out), n, batch, direction,
                                    ctypes.byref(plan) if plan is not None else None,
                                    _stream(stream, inp, out)))


def make_plan(log2_n1, radix_a, radix_b, tile_a=16, tile_b=16):
    return FftPlan(log2_n1, radix_a, radix_b, tile_a, tile_b)


def fft_plan_valid(n, plan) -> bool:
    return _tl("ppx_fft_plan_valid")(n, ctypes.byref(plan)) == 0


def enumerate_fft_plans(n):
    f = _tl("ppx_enumerate_fft_plans")
    cnt = _check(f(n, None, 0))
    arr = (FftPlan * max(cnt, 1))()
    _check(f(n, arr, cnt))
    return [FftPlan(*arr[i].as_tuple()) for i in range(cnt)]


def default_fft_plan(n):
    p = FftPlan()
    _check(_tl("ppx_default_fft_plan")(n, ctypes.byref(p)))
    return p


def tune_fft_large(n, batch, method, max_evals=0, reps=100, trace_cap=None):
    """Returns (plan, best_us, evals_used, [(plan, us) timed in order]); the
    trace holds every timed plan unless trace_cap is smaller."""
    if trace_cap is None:
        trace_cap = max(1, len(enumerate_fft_plans(n)))
    best = FftPlan()
    us = ctypes.c_double(0.0)
    ev = ctypes.c_int(0)
    tp = (FftPlan * trace_cap)()
    tu = (ctypes.c_double * trace_cap)()
    cnt = _check(_tl("ppx_tune_large_trace")(n, batch, method, max_evals, reps, ctypes.byref(best),
                                              ctypes.byref(us), ctypes.byref(ev), tp, tu, trace_cap))
    trace = [(FftPlan(*tp[i].as_tuple()), tu[i]) for i in range(min(cnt, trace_cap))]
    return best, us.value, ev.value, trace


def occupancy(model, res):
    b, w = ctypes.c_int32(0), ctypes.c_int32(0)
    _tl("ppx_occupancy")(ctypes.byref(model), ctypes.byref(res), ctypes.byref(b), ctypes.byref(w))
    return b.value, w.value


def device_model_gfx950():
    m = DeviceModel()
    _check(_tl("ppx_device_model_gfx950")(ctypes.byref(m)))
    return m


def analytical_pick(model, cands, resources, batch, flags=0):
    n = len(cands)
    ca = (Config * n)(*cands)
    ra = (Resource * n)(*resources)
    k = ctypes.c_int(-1)
    _check(_tl("ppx_analytical_pick")(ctypes.byref(model), ca, ra, n, batch, flags, ctypes.byref(k)))
    return k.value


def analytical_select(op, dtype, n, batch, cands):
    """Index of the library's analytical choice among cands (ppx_tune.h)."""
    ca = (Config * len(cands))(*cands)
    k = ctypes.c_int(-1)
    _check(_tl("ppx_analytical_select")(op, dtype, n, batch, ca, len(cands), ctypes.byref(k)))
    return k.value


def bo_search(cands, evaluate, max_evals=0, n_init=0, patience=0, min_rel=0.01, seed=0):
    """Bayesian search with a Python evaluator evaluate(Config) -> cost (<0 = failed).
    Returns (best_index, order, values)."""
    n = len(cands)
    ca = (Config * n)(*cands)
    order = (ctypes.c_int * n)()
    vals = (ctypes.c_double * n)()
    used, best = ctypes.c_int(0), ctypes.c_int(-1)
    errors = []

    def _cb(cp, _user):
        try:
            return float(evaluate(cp.contents))
        except Exception as e:  # a failing evaluator is a failed run
            errors.append(e)
            return -1.0
    cb = EVAL_FN(_cb)
    _check(_tl("ppx_bo_search")(ca, n, cb, None, max_evals, n_init, patience, min_rel, seed,
                                order, vals, ctypes.byref(used), ctypes.byref(best)))
    k = used.value
    return best.value, list(order[:k]), list(vals[:k])


def gp_posterior(X, y, lengthscales, sigma_f2, noise2, Xq):
    import numpy as np
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xq = np.ascontiguousarray(Xq, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    ls = np.ascontiguousarray(lengthscales, dtype=np.float64)
    n, d = X.shape
    m = Xq.shape[0]
    mu = np.empty(m)
    var = np.empty(m)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    _check(_tl("ppx_gp_posterior")(dp(X), dp(y), n, d, dp(ls), sigma_f2, noise2, dp(Xq), m,
                                   dp(mu), dp(var)))
    return mu, var


def expected_improvement(mu, sigma, best):
    return _tl("ppx_expected_improvement")(mu, sigma, best)


def tune_ex(op, dtype, n, batch, method, max_evals=0, algo=-1, reps=0, trace_cap=256):
    rep = TuneReport()
    tc = (Config * trace_cap)()
    tu = (ctypes.c_double * trace_cap)()
    rep.trace_cfg = tc
    rep.trace_us = tu
    rep.trace_cap = trace_cap
    _check(_tl("ppx_tune_ex")(op, dtype, n, batch, method, max_evals, algo, reps, ctypes.byref(rep)))
    k = min(rep.evals_used if method != TUNE_ANALYTICAL else 1, trace_cap)
    return rep, [(tc[i], tu[i]) for i in range(k)]


def time_config(op, dtype, n, batch, cfg, reps=0):
    us = ctypes.c_double(0)
    _check(_tl("ppx_time_config")(op, dtype, n, batch, ctypes.byref(cfg), reps, ctypes.byref(us)))
    return us.value


def kernel_resources(op, dtype, n, cfg):
    r = Resource()
    _check(_tl("ppx_kernel_resources")(op, dtype, n, ctypes.byref(cfg), ctypes.byref(r)))
    return r


def stream_reference(inputs, out, nbytes, stream=None):
    """Plain streaming kernel over len(inputs) input arrays and one output of
    nbytes bytes each (the practical bandwidth ceiling of a call with that
    many input streams); torch tensors or raw device pointers."""
    arr = (ctypes.c_void_p * len(inputs))(*[_ptr(t) for t in inputs])
    _check(_tl("ppx_stream_reference")(arr, len(inputs), _ptr(out), nbytes, _stream(stream, out)))


def load_tune_cache(path):
    return _check(_tl("ppx_tune_cache_load")(os.fsencode(path)))


def save_tune_cache(path):
    _check(_tl("ppx_tune_cache_save")(os.fsencode(path)))


def clear_tune_cache():
    _tl("ppx_tune_cache_clear")()


def tuned_fft_plan(n):
    """The tuned large-FFT plan recorded for n, or None."""
    p = FftPlan()
    f = lib().ppx_tuned_fft_plan
    f.argtypes, f.restype = [ctypes.c_int64, ctypes.POINTER(FftPlan)], ctypes.c_int
    return p if f(n, ctypes.byref(p)) == OK else None


def tuned_config(op, dtype, n, algo=-1):
    c = Config()
    if _tl("ppx_tuned_config")(op, dtype, n, algo, ctypes.byref(c)) != OK:
        return None
    return c


def phi(efficiencies):
    """Harmonic mean of per-size efficiencies (Sec. VI's performance-portability
    metric): |C| / sum 1/e_i."""
    e = [float(v) for v in efficiencies]
    return len(e) / sum(1.0 / v for v in e)


# ---------------------------------------------------------------- mixed launch

class Job(ctypes.Structure):
    """ppx_job: one whole batched call inside a mixed launch."""
    _fields_ = [("op", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("n", ctypes.c_int64), ("batch", ctypes.c_int64),
                ("in_", ctypes.c_void_p), ("b", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("d", ctypes.c_void_p), ("out", ctypes.c_void_p)]


def make_job(op, dtype, n, batch, inp, out, direction=-1, algo=0, b=None, c=None, d=None):
    return Job(op, dtype, direction, algo, n, batch, _ptr(inp), _ptr(b), _ptr(c), _ptr(d),
               _ptr(out))


def launch_mixed(jobs, stream=None):
    """One fused launch over a list of Job (see include/ppx.h)."""
    L = lib()
    f = L.launch_mixed
    if not getattr(f, "_ppx_typed", False):
        f.argtypes = [ctypes.POINTER(Job), ctypes.c_int, ctypes.c_void_p]
        f.restype = ctypes.c_int
        f._ppx_typed = True
    arr = (Job * len(jobs))(*jobs)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(f(arr, len(jobs), stream))


NOALLOC_MAX_JOBS, NOALLOC_MAX_TILES = 256, 262144
MIXED_DIRECT_ELEMS = 1 << 22  # a persistent-configured job this large runs as its own call
PIPE_FLAG = {0: 2, 1: 2, 2: 8}  # the persistent flag of each op's algo codes (FFT, scan, tridiagonal)


def mixed_job_is_direct(op, n, batch, cfg):
    """Whether launch_mixed runs a job with resolved configuration cfg as its
    own single call (see PPX_MIXED_DIRECT_ELEMS in include/ppx.h)."""
    return bool(cfg.algo & PIPE_FLAG[op]) and n * batch >= MIXED_DIRECT_ELEMS


def launch_mixed_noalloc(jobs, stream=None):
    """launch_mixed with its tables in the library's static device array (no
    allocation; see include/ppx.h)."""
    f = lib().launch_mixed_noalloc
    if not getattr(f, "_ppx_typed", False):
        f.argtypes = [ctypes.POINTER(Job), ctypes.c_int, ctypes.c_void_p]
        f.restype = ctypes.c_int
        f._ppx_typed = True
    arr = (Job * len(jobs))(*jobs)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(f(arr, len(jobs), stream))


MIXED_ARG_JOBS = 32  # most jobs of one family a launch passes in kernel arguments


def mixed_argument_launch(jobs):
    """Whether launch_mixed passes these jobs' records in the kernel
    arguments (True) or uses the device tables and persistent kernels."""
    f = lib().ppx_mixed_argument_launch
    if not getattr(f, "_ppx_typed", False):
        f.argtypes = [ctypes.POINTER(Job), ctypes.c_int]
        f.restype = ctypes.c_int
        f._ppx_typed = True
    arr = (Job * len(jobs))(*jobs)
    return _check(f(arr, len(jobs))) == 1


def mixed_tile_config(job):
    """How launch_mixed cuts a Job: (problems per tile, Config whose
    arithmetic the tiles follow)."""
    f = lib().ppx_mixed_tile_config
    if not getattr(f, "_ppx_typed", False):
        f.argtypes = [ctypes.POINTER(Job), ctypes.POINTER(Config)]
        f.restype = ctypes.c_int
        f._ppx_typed = True
    c = Config()
    per = _check(f(ctypes.byref(job), ctypes.byref(c)))
    return per, c


# ---------------------------------------------------------------- serving
# (declared in include/ppx_serve.h)

SERVE_FUSED, SERVE_PER_REQUEST, SERVE_NULL_DEVICE, SERVE_ONLINE_TUNE = 0, 1, 2, 4
JOB_SCAN_INCLUSIVE, JOB_SCAN_EXCLUSIVE = 0, 1  # the algo field of a scan job


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("out", ctypes.c_void_p), ("arrival_us", ctypes.c_double),
                ("admit_us", ctypes.c_double), ("complete_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "admitted", "completed", "released",
                                              "launches", "budget_bytes", "used_bytes",
                                              "peak_used_bytes")] + \
               [("max_inflight_seen", ctypes.c_int32), ("pending", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("job", Job), ("arrival_us", ctypes.c_double)]


def _sl(name, argtypes):
    f = getattr(lib(), name)
    if not getattr(f, "_ppx_typed", False):
        f.argtypes = argtypes
        f.restype = ctypes.c_int
        f._ppx_typed = True
    return f


class Server:
    """Continuous-batching request loop (include/ppx_serve.h)."""

    def __init__(self, budget_bytes, max_inflight=2, flags=SERVE_FUSED):
        self._h = ctypes.c_void_p()
        _check(_sl("ppx_server_create", [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)])(
            budget_bytes, max_inflight, flags, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _sl("ppx_server_destroy", [ctypes.c_void_p])(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, job):
        i = ctypes.c_int64(0)
        _check(_sl("ppx_server_submit", [ctypes.c_void_p, ctypes.POINTER(Job),
                                         ctypes.POINTER(ctypes.c_int64)])(
            self._h, ctypes.byref(job), ctypes.byref(i)))
        return i.value

    def progress(self):
        k = ctypes.c_int(0)
        _check(_sl("ppx_server_progress", [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)])(
            self._h, ctypes.byref(k)))
        return k.value

    def poll(self, cap=1024):
        arr = (Completion * cap)()
        k = ctypes.c_int(0)
        _check(_sl("ppx_server_poll", [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int)])(
            self._h, arr, cap, ctypes.byref(k)))
        return [arr[i] for i in range(k.value)]

    def release(self, job_id):
        _check(_sl("ppx_server_release", [ctypes.c_void_p, ctypes.c_int64])(self._h, job_id))

    def read(self, job_id, host_array):
        import numpy as np
        assert isinstance(host_array, np.ndarray) and host_array.flags.c_contiguous
        _check(_sl("ppx_server_read", [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_int64])(
            self._h, job_id, host_array.ctypes.data, host_array.nbytes))
        return host_array

    def stats(self):
        st = ServerStats()
        _check(_sl("ppx_server_stats_get", [ctypes.c_void_p, ctypes.POINTER(ServerStats)])(
            self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def online_stats(self):
        """(sessions, evaluation launches, sessions whose search has stopped)."""
        ses, ev, conv = ctypes.c_int(0), ctypes.c_int64(0), ctypes.c_int(0)
        _check(_sl("ppx_server_online_stats", [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)])(
            self._h, ctypes.byref(ses), ctypes.byref(ev), ctypes.byref(conv)))
        return dict(sessions=ses.value, evaluations=ev.value, converged=conv.value)

    def replay(self, requests, auto_release=True):
        """requests: list of (Job, arrival_us) sorted by arrival; returns a list
        of Completion in request order."""
        n = len(requests)
        arr = (Request * n)(*[Request(j, t) for j, t in requests])
        out = (Completion * n)()
        _check(_sl("ppx_serve_replay", [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(Completion)])(
            self._h, arr, n, 1 if auto_release else 0, out))
        return [out[i] for i in range(n)]
