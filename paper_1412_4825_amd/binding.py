"""ctypes binding of libbrng.so: the C functions under the same names.

Only argument marshalling happens here: every deviate is produced by the HIP
kernels behind the C interface (include/brng.h).  Device arrays are passed as
torch tensors (their data_ptr) or raw integer addresses; torch is used only
for device memory and streams.  If the library is missing this module raises
at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbrng.so")

BRNG_OK, BRNG_E_ARG, BRNG_E_NOMEM, BRNG_E_HIP, BRNG_E_KIND_DISABLED, BRNG_E_BUSY, BRNG_E_UNSUPPORTED, BRNG_E_TOO_LARGE = range(8)
STATIC_SCRATCH_MB = 32
BRNG_U, BRNG_N, BRNG_E, BRNG_U64 = 0, 1, 2, 3
BRNG_F32, BRNG_F64 = 0, 1
BRNG_LAYOUT_CHAINS, BRNG_LAYOUT_ITEMS = 0, 1
BRNG_MODEL_TRIANGLE_F64, BRNG_MODEL_NORMEXP, BRNG_MODEL_GAMMA_CHAIN, BRNG_MODEL_LDA, BRNG_MODEL_EXP_CHAIN = range(5)
BRNG_FLAG_RESUME = 1
BRNG_LDAF_COUNTS_VALID = 1
UNIT_WIDTH = 64
BATCH_MAX = 4096
WINDOW_ALIGN = 256
WINDOW_MIN = 512

EXPORTS = [
    "brng_create", "brng_destroy", "brng_fill_base", "brng_step_uniform", "brng_step_normal",
    "brng_step_exp", "brng_step_gamma", "brng_step_laplace", "brng_step_weibull", "brng_step_poisson",
    "brng_step_binomial", "brng_step_multinomial",
    "brng_step_dirichlet", "brng_run_gibbs", "brng_run_gibbs_static", "brng_run_lda_full",
    "brng_lda_full_units",
    "brng_sort_by_length", "brng_get_cursors", "brng_set_cursors", "brng_get_window",
    "brng_get_info", "brng_set_launch", "brng_time_next_launch", "brng_status_string",
    "brng_last_hip_error",
    "brng_convert", "brng_serve_open", "brng_serve_now", "brng_serve_submit",
    "brng_serve_progress", "brng_serve_poll", "brng_serve_stats_get", "brng_serve_close",
]


class brng_config(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("n_chains", C.c_uint32),
        ("layout", C.c_uint32),
        ("window", C.c_uint32 * 4),
        ("prec", C.c_int32),
        ("hip_stream", C.c_void_p),
    ]


class brng_gibbs_desc(C.Structure):
    _fields_ = [
        ("model", C.c_int32),
        ("n_chains", C.c_uint32),
        ("unit_base", C.c_uint32),
        ("flags", C.c_uint32),
        ("seed", C.c_uint64),
        ("max_steps", C.c_int32),
        ("pad0", C.c_int32),
        ("d_steps", C.c_void_p),
        ("d_perm", C.c_void_p),
        ("d_state", C.c_void_p),
        ("d_trace", C.c_void_p),
        ("d_trace2", C.c_void_p),
        ("trace_stride", C.c_int64),
        ("d_offsets", C.c_void_p),
        ("d_ntok", C.c_void_p),
        ("d_sums", C.c_void_p),
    ]


class brng_lda_full_desc(C.Structure):
    _fields_ = [
        ("n_docs", C.c_uint32),
        ("n_topics", C.c_uint32),
        ("n_vocab", C.c_uint32),
        ("sweeps", C.c_uint32),
        ("n_tokens", C.c_int32),
        ("alpha", C.c_float),
        ("beta", C.c_float),
        ("flags", C.c_uint32),
        ("d_doc_offsets", C.c_void_p),
        ("d_words", C.c_void_p),
        ("d_z", C.c_void_p),
        ("d_ndk", C.c_void_p),
        ("d_nkw", C.c_void_p),
        ("d_theta", C.c_void_p),
        ("d_phi", C.c_void_p),
    ]


class brng_serve_config(C.Structure):
    _fields_ = [
        ("hbm_budget", C.c_uint64),
        ("max_active", C.c_uint32),
        ("tick_steps", C.c_uint32),
        ("tick_sweeps", C.c_uint32),
        ("window", C.c_uint32 * 4),
        ("max_bypass_ms", C.c_uint32),
        ("hip_stream", C.c_void_p),
    ]


class brng_serve_done(C.Structure):
    _fields_ = [
        ("ticket", C.c_uint64),
        ("t_arrive_ns", C.c_uint64),
        ("t_admit_ns", C.c_uint64),
        ("t_done_ns", C.c_uint64),
        ("status", C.c_int32),
        ("pad", C.c_int32),
    ]


class brng_serve_stats(C.Structure):
    _fields_ = [
        ("waiting", C.c_uint32),
        ("active", C.c_uint32),
        ("ticks_in_flight", C.c_uint32),
        ("pad", C.c_uint32),
        ("bytes_in_use", C.c_uint64),
        ("bytes_peak", C.c_uint64),
        ("ticks", C.c_uint64),
        ("completed", C.c_uint64),
    ]


class BrngError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.brng_status_string(status).decode() if _lib is not None else str(status)
        extra = ""
        if status == BRNG_E_HIP and _lib is not None:
            extra = " (hipError %d)" % _lib.brng_last_hip_error()
        super().__init__("%s: %s%s" % (where, msg, extra))
        self.status = status


def _load():
    # PyTorch brings its own HIP runtime (same soname as the system one).  It
    # is loaded first so that this library binds to it: a process must not
    # hold two HIP runtimes, or the second finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libbrng.so not built (expected at %s); run `python -m paper_1412_4825_amd.build`"
            % LIB_PATH
        )
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.brng_create.argtypes = [C.POINTER(brng_config), C.POINTER(vp)]
    L.brng_destroy.argtypes = [vp]
    L.brng_fill_base.argtypes = [vp, C.c_int32]
    L.brng_step_uniform.argtypes = [vp, vp, vp, vp]
    L.brng_step_normal.argtypes = [vp, vp, vp, vp]
    L.brng_step_exp.argtypes = [vp, vp, vp]
    L.brng_step_gamma.argtypes = [vp, vp, vp]
    L.brng_step_laplace.argtypes = [vp, vp, vp, vp]
    L.brng_step_weibull.argtypes = [vp, vp, vp, vp]
    L.brng_step_poisson.argtypes = [vp, vp, vp]
    L.brng_step_binomial.argtypes = [vp, vp, vp, vp]
    L.brng_step_multinomial.argtypes = [vp, vp, vp, vp, vp]
    L.brng_step_dirichlet.argtypes = [vp, vp, vp, vp]
    L.brng_run_gibbs.argtypes = [vp, C.POINTER(brng_gibbs_desc), C.c_uint32]
    L.brng_run_gibbs_static.argtypes = [C.POINTER(brng_gibbs_desc), vp, C.c_int32, vp]
    L.brng_run_lda_full.argtypes = [vp, C.POINTER(brng_lda_full_desc)]
    L.brng_lda_full_units.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
    L.brng_lda_full_units.restype = C.c_uint64
    L.brng_sort_by_length.argtypes = [C.c_uint32, vp, vp]
    L.brng_get_cursors.argtypes = [vp, vp]
    L.brng_set_cursors.argtypes = [vp, vp]
    L.brng_get_window.argtypes = [vp, C.c_int32, C.c_uint32, vp, C.c_uint32,
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]
    L.brng_get_info.argtypes = [vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
    L.brng_set_launch.argtypes = [vp, C.c_int32, C.c_int32]
    L.brng_time_next_launch.argtypes = [vp, vp, vp]
    L.brng_convert.argtypes = [C.c_int32, vp, C.c_uint64, vp, vp]
    L.brng_serve_open.argtypes = [C.POINTER(brng_serve_config), C.POINTER(vp)]
    L.brng_serve_now.argtypes = []
    L.brng_serve_now.restype = C.c_uint64
    L.brng_serve_submit.argtypes = [vp, C.POINTER(brng_gibbs_desc), C.c_uint64,
                                    C.POINTER(C.c_uint64)]
    L.brng_serve_progress.argtypes = [vp, C.c_int32]
    L.brng_serve_poll.argtypes = [vp, C.POINTER(brng_serve_done), C.c_uint32,
                                  C.POINTER(C.c_uint32)]
    L.brng_serve_stats_get.argtypes = [vp, C.POINTER(brng_serve_stats)]
    L.brng_serve_close.argtypes = [vp]
    L.brng_status_string.argtypes = [C.c_int32]
    L.brng_status_string.restype = C.c_char_p
    L.brng_last_hip_error.argtypes = []
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is C.c_int:  # ctypes default
            f.restype = C.c_int32
    return L


_lib = _load()


def lib():
    return _lib


def _check(status: int, where: str):
    if status != BRNG_OK:
        raise BrngError(status, where)


def _ptr(x):
    """Device/host address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError("unsupported array type %r" % type(x))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# the C functions
# ---------------------------------------------------------------------------

def brng_create(seed: int, n_chains: int, window, layout: int = BRNG_LAYOUT_CHAINS,
                prec: int = BRNG_F32, stream=None) -> int:
    cfg = brng_config()
    cfg.seed = seed
    cfg.n_chains = n_chains
    cfg.layout = layout
    for k in range(4):
        cfg.window[k] = int(window[k])
    cfg.prec = prec
    cfg.hip_stream = _stream_handle(stream)
    out = C.c_void_p()
    _check(_lib.brng_create(C.byref(cfg), C.byref(out)), "brng_create")
    return out.value


def brng_destroy(ctx: int) -> None:
    _check(_lib.brng_destroy(ctx), "brng_destroy")


def brng_fill_base(ctx: int, kind: int) -> None:
    _check(_lib.brng_fill_base(ctx, kind), "brng_fill_base")


def brng_step_uniform(ctx, a, b, out) -> None:
    _check(_lib.brng_step_uniform(ctx, _ptr(a), _ptr(b), _ptr(out)), "brng_step_uniform")


def brng_step_normal(ctx, mu, sigma, out) -> None:
    _check(_lib.brng_step_normal(ctx, _ptr(mu), _ptr(sigma), _ptr(out)), "brng_step_normal")


def brng_step_exp(ctx, lam, out) -> None:
    _check(_lib.brng_step_exp(ctx, _ptr(lam), _ptr(out)), "brng_step_exp")


def brng_step_gamma(ctx, alpha, out) -> None:
    _check(_lib.brng_step_gamma(ctx, _ptr(alpha), _ptr(out)), "brng_step_gamma")


def brng_step_laplace(ctx, mu, b, out) -> None:
    _check(_lib.brng_step_laplace(ctx, _ptr(mu), _ptr(b), _ptr(out)), "brng_step_laplace")


def brng_step_weibull(ctx, lam, k, out) -> None:
    _check(_lib.brng_step_weibull(ctx, _ptr(lam), _ptr(k), _ptr(out)), "brng_step_weibull")


def brng_step_poisson(ctx, lam, out) -> None:
    _check(_lib.brng_step_poisson(ctx, _ptr(lam), _ptr(out)), "brng_step_poisson")


def brng_step_binomial(ctx, n, p, out) -> None:
    _check(_lib.brng_step_binomial(ctx, _ptr(n), _ptr(p), _ptr(out)), "brng_step_binomial")


def brng_step_multinomial(ctx, offsets, n, w, out) -> None:
    _check(_lib.brng_step_multinomial(ctx, _ptr(offsets), _ptr(n), _ptr(w), _ptr(out)),
           "brng_step_multinomial")


def brng_step_dirichlet(ctx, offsets, alpha, out) -> None:
    _check(_lib.brng_step_dirichlet(ctx, _ptr(offsets), _ptr(alpha), _ptr(out)),
           "brng_step_dirichlet")


def gibbs_desc(model: int, n_chains: int, state, *, max_steps: int, seed: int,
               unit_base: int = 0, flags: int = 0, steps=None, perm=None, trace=None,
               trace2=None, trace_stride: int = 0, offsets=None, ntok=None,
               sums=None) -> brng_gibbs_desc:
    d = brng_gibbs_desc()
    d.model = model
    d.n_chains = n_chains
    d.unit_base = unit_base
    d.flags = flags
    d.seed = seed
    d.max_steps = max_steps
    d.d_steps = _ptr(steps)
    d.d_perm = _ptr(perm)
    d.d_state = _ptr(state)
    d.d_trace = _ptr(trace)
    d.d_trace2 = _ptr(trace2)
    d.trace_stride = trace_stride
    d.d_offsets = _ptr(offsets)
    d.d_ntok = _ptr(ntok)
    d.d_sums = _ptr(sums)
    return d


def brng_run_gibbs(ctx: int, descs) -> None:
    if isinstance(descs, brng_gibbs_desc):
        descs = [descs]
    arr = (brng_gibbs_desc * len(descs))(*descs)
    _check(_lib.brng_run_gibbs(ctx, arr, len(descs)), "brng_run_gibbs")


def brng_run_gibbs_static(desc: brng_gibbs_desc, window, wpb: int = 4, stream=None) -> None:
    w = (C.c_uint32 * 4)(*[int(x) for x in window])
    _check(_lib.brng_run_gibbs_static(C.byref(desc), w, wpb, _stream_handle(stream)),
           "brng_run_gibbs_static")


def brng_sort_by_length(steps) -> np.ndarray:
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    perm = np.zeros(steps.size, dtype=np.int32)
    _check(_lib.brng_sort_by_length(steps.size, steps.ctypes.data, perm.ctypes.data),
           "brng_sort_by_length")
    return perm


def brng_get_info(ctx: int):
    nu = C.c_uint32()
    w = (C.c_uint32 * 4)()
    _check(_lib.brng_get_info(ctx, C.byref(nu), w), "brng_get_info")
    return nu.value, [w[k] for k in range(4)]


def brng_get_cursors(ctx: int) -> np.ndarray:
    nu, _ = brng_get_info(ctx)
    out = np.zeros((nu, 4), dtype=np.uint64)
    _check(_lib.brng_get_cursors(ctx, out.ctypes.data), "brng_get_cursors")
    return out


def brng_set_cursors(ctx: int, cursors) -> None:
    cur = np.ascontiguousarray(cursors, dtype=np.uint64)
    nu, _ = brng_get_info(ctx)
    if cur.shape != (nu, 4):
        raise ValueError("cursors must have shape (%d, 4)" % nu)
    _check(_lib.brng_set_cursors(ctx, cur.ctypes.data), "brng_set_cursors")


def brng_get_window(ctx: int, kind: int, unit: int):
    """(pool index of element 0, valid length, entries as numpy)."""
    _, w = brng_get_info(ctx)
    cap = w[kind]
    out = np.zeros(cap, dtype=np.float64 if kind == BRNG_U64 else np.float32)
    base, ln = C.c_uint64(), C.c_uint32()
    _check(_lib.brng_get_window(ctx, kind, unit, out.ctypes.data, cap, C.byref(base), C.byref(ln)),
           "brng_get_window")
    return base.value, ln.value, out


def brng_set_launch(ctx: int, waves_per_block: int) -> None:
    _check(_lib.brng_set_launch(ctx, waves_per_block, 0), "brng_set_launch")


def brng_lda_full_units(n_topics: int, n_vocab: int, n_docs: int) -> int:
    """Items (units) a full-LDA corpus of this shape uses."""
    return int(_lib.brng_lda_full_units(n_topics, n_vocab, n_docs))


def brng_run_lda_full(ctx: int, n_topics: int, n_vocab: int, sweeps: int, alpha: float,
                      beta: float, doc_offsets, words, z, ndk, nkw, theta, phi,
                      counts_valid: bool = False) -> None:
    """Full LDA sweeps over the corpus (device int32 doc_offsets, words, z;
    outputs ndk, nkw, theta, phi); counts_valid skips the recount of ndk and
    nkw from z."""
    d = brng_lda_full_desc()
    d.flags = BRNG_LDAF_COUNTS_VALID if counts_valid else 0
    d.n_docs = int(doc_offsets.numel()) - 1
    d.n_topics, d.n_vocab, d.sweeps = int(n_topics), int(n_vocab), int(sweeps)
    d.n_tokens = int(words.numel()) if words is not None else 0
    d.alpha, d.beta = float(alpha), float(beta)
    d.d_doc_offsets, d.d_words, d.d_z = _ptr(doc_offsets), _ptr(words), _ptr(z)
    d.d_ndk, d.d_nkw, d.d_theta, d.d_phi = _ptr(ndk), _ptr(nkw), _ptr(theta), _ptr(phi)
    _check(_lib.brng_run_lda_full(ctx, C.byref(d)), "brng_run_lda_full")


def brng_time_next_launch(ctx: int, start=None, stop=None) -> None:
    """Record two timing events (torch.cuda.Event with enable_timing, or raw
    hipEvent_t handles) at the start and end of the next plain chain launch;
    no events clears a pending pair."""
    def handle(e):
        if e is None:
            return None
        if not hasattr(e, "cuda_event"):
            return int(e)
        if not e.cuda_event:  # torch creates the HIP event at its first record
            e.record()
        return e.cuda_event
    _check(_lib.brng_time_next_launch(ctx, handle(start), handle(stop)), "brng_time_next_launch")


def brng_convert(kind: int, words, n_words: int, out, stream=None) -> None:
    _check(_lib.brng_convert(kind, _ptr(words), n_words, _ptr(out), _stream_handle(stream)),
           "brng_convert")


def brng_status_string(status: int) -> str:
    return _lib.brng_status_string(status).decode()


# ---------------------------------------------------------------------------
# served form
# ---------------------------------------------------------------------------

def brng_serve_open(hbm_budget: int, window, *, max_active: int = 64, tick_steps: int = 64,
                    tick_sweeps: int = 2, max_bypass_ms: int = 0, stream=None) -> int:
    cfg = brng_serve_config()
    cfg.hbm_budget = hbm_budget
    cfg.max_bypass_ms = max_bypass_ms
    cfg.max_active = max_active
    cfg.tick_steps = tick_steps
    cfg.tick_sweeps = tick_sweeps
    for k in range(4):
        cfg.window[k] = int(window[k])
    cfg.hip_stream = _stream_handle(stream)
    out = C.c_void_p()
    _check(_lib.brng_serve_open(C.byref(cfg), C.byref(out)), "brng_serve_open")
    return out.value


def brng_serve_now() -> int:
    return int(_lib.brng_serve_now())


def brng_serve_submit(srv: int, desc: brng_gibbs_desc, t_arrive_ns: int = 0) -> int:
    t = C.c_uint64()
    _check(_lib.brng_serve_submit(srv, C.byref(desc), t_arrive_ns, C.byref(t)),
           "brng_serve_submit")
    return t.value


def brng_serve_progress(srv: int, wait: bool = False) -> None:
    _check(_lib.brng_serve_progress(srv, 1 if wait else 0), "brng_serve_progress")


def brng_serve_poll(srv: int, cap: int = 256):
    """Finished requests as a list of dicts (ticket, t_arrive_ns, t_admit_ns,
    t_done_ns, status)."""
    buf = (brng_serve_done * cap)()
    n = C.c_uint32()
    _check(_lib.brng_serve_poll(srv, buf, cap, C.byref(n)), "brng_serve_poll")
    return [{f: getattr(buf[i], f) for f, _ in brng_serve_done._fields_ if f != "pad"}
            for i in range(n.value)]


def brng_serve_stats_get(srv: int) -> dict:
    o = brng_serve_stats()
    _check(_lib.brng_serve_stats_get(srv, C.byref(o)), "brng_serve_stats_get")
    return {f: getattr(o, f) for f, _ in brng_serve_stats._fields_ if f != "pad"}


def brng_serve_close(srv: int) -> None:
    _check(_lib.brng_serve_close(srv), "brng_serve_close")
