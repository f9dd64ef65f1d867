"""Plain CPU oracle for the varying-parameter base-pool RNG (double precision).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never does, and it shares no code with it.

The arithmetic lives in ``brng_oracle.c`` (scalar C, FP64, one file); this
module builds it with gcc when needed and marshals numpy arrays through
ctypes.  Every function documents the passage of Mahani & Sharabiani (arXiv
1412.4825) it follows; see the C file's header for the stream contract.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against values fixed by the paper or by mathematics (closed forms, library
distributions, an independent Philox implementation, brute force).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brng_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KIND_U, KIND_N, KIND_E, KIND_U64 = 0, 1, 2, 3
UNIT_WIDTH = 64  # chains per unit: the stream contract's grouping


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_u8p = C.POINTER(C.c_uint8)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)
_i32p = C.POINTER(C.c_int32)
_dp = C.POINTER(C.c_double)


def _declare(L):
    L.or_philox4x32.argtypes = [_u32p, _u32p, C.c_int, _u32p]
    L.or_block_words.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, _u32p]
    L.or_u32.argtypes = [C.c_uint32]
    L.or_u32.restype = C.c_double
    L.or_u64.argtypes = [C.c_uint32, C.c_uint32]
    L.or_u64.restype = C.c_double
    L.or_entry.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64]
    L.or_entry.restype = C.c_double
    L.or_entries.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, _dp]
    L.or_words.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64, _u32p]
    L.or_tol.argtypes = [C.c_double]
    L.or_tol.restype = C.c_double
    L.or_u32_many.argtypes = [_u32p, C.c_uint64, _dp]
    L.or_convert.argtypes = [C.c_int, _u32p, C.c_uint64, _dp]
    L.or_step_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _u64p, _dp, _dp, _dp, _dp]
    L.or_step_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _dp, _dp, _dp]
    L.or_step_exp.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _dp, _dp]
    L.or_step_laplace.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _dp,
                                  _dp, _dp]
    L.or_step_weibull.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _dp,
                                  _dp, _dp]
    L.or_step_gamma.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _dp, _dp, _dp, _i32p, _i32p]
    L.or_step_poisson.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _dp, _i32p, _dp]
    L.or_step_binomial.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _i32p, _dp, _i32p,
                                   _dp]
    L.or_step_multinomial.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u64p, _i32p, _i32p,
                                      _dp, _i32p, _dp]
    L.or_step_dirichlet.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, _u64p, _i32p, _dp, _dp, _dp, _dp]
    L.or_dirichlet_blocks.argtypes = [C.c_uint64, C.c_uint32, C.c_int32, C.c_int32, _u64p, _dp, _dp, _dp,
                                      _dp]
    L.or_multinomial.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, _u64p, _i32p, _i32p, _dp, _i32p]
    L.or_triangle.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _dp, _dp, _u64p, _dp, _dp, _dp, _dp]
    L.or_normexp.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _dp, _u64p, _dp, _dp, _dp, _dp]
    L.or_expchain.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, _dp, _u64p, _dp, _dp]
    L.or_gamma_chain.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _i32p, _i32p, _dp, _u64p, _dp, _dp, _dp,
                                 _i32p, _i32p]
    L.or_normexp_replay.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                    _dp, _dp, _u64p, _dp, _dp, _dp, _dp, _dp, _dp]
    L.or_expchain_replay.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                     _dp, _u64p, _dp, _dp, _dp, _dp]
    L.or_gamma_chain_replay.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _i32p, _i32p, _dp,
                                        _u64p, _dp, _dp, _dp, _i32p, _i32p]
    L.or_lda.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, _i32p, _i32p, C.c_uint32, _i32p, _u64p, _dp, _dp, _i32p, _dp, _dp]


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _n_units(n, width=UNIT_WIDTH):
    return (n + width - 1) // width


def new_cursors(n_units: int) -> np.ndarray:
    """Four pool counters per unit, all at zero (constructor, Sec. 2.2)."""
    return np.zeros((n_units, 4), dtype=np.uint64)


# --------------------------------------------------------------------------
# Core engine and conversions
# --------------------------------------------------------------------------

def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32(_p(c, _u32p), _p(k, _u32p), int(rounds), _p(out, _u32p))
    return out


def words(seed: int, unit: int, kind: int, block0: int, nblocks: int) -> np.ndarray:
    """Raw Philox words of pool blocks [block0, block0 + nblocks)."""
    out = np.zeros(4 * nblocks, dtype=np.uint32)
    lib().or_words(seed, unit, kind, block0, nblocks, _p(out, _u32p))
    return out


def u32(w: int) -> float:
    return lib().or_u32(int(w))


def u64(wa: int, wb: int) -> float:
    return lib().or_u64(int(wa), int(wb))


def entries(seed: int, unit: int, kind: int, j0: int, n: int) -> np.ndarray:
    """Pool entries [j0, j0 + n) of (seed, unit, kind), in double precision."""
    out = np.zeros(n, dtype=np.float64)
    lib().or_entries(seed, unit, kind, j0, n, _p(out, _dp))
    return out


def tol(m) -> np.ndarray:
    """max(4 ulp32(M), 1e-6 M) elementwise."""
    f = lib().or_tol
    return np.array([f(float(x)) for x in np.ravel(m)]).reshape(np.shape(m))


# --------------------------------------------------------------------------
# One call per chain (the one-at-a-time scenario, Sec. 1)
# --------------------------------------------------------------------------

def step_uniform(seed, cursors, a, b, kind=KIND_U, width=UNIT_WIDTH, unit0=0):
    a, b = _d(a), _d(b)
    n = a.size
    out, t = np.zeros(n), np.zeros(n)
    lib().or_step_uniform(seed, unit0, n, width, kind, _p(cursors, _u64p), _p(a, _dp), _p(b, _dp),
                          _p(out, _dp), _p(t, _dp))
    return out, t


def step_normal(seed, cursors, mu, sigma, width=UNIT_WIDTH, unit0=0):
    mu, sigma = _d(mu), _d(sigma)
    n = mu.size
    out, t = np.zeros(n), np.zeros(n)
    lib().or_step_normal(seed, unit0, n, width, _p(cursors, _u64p), _p(mu, _dp), _p(sigma, _dp),
                         _p(out, _dp), _p(t, _dp))
    return out, t


def step_exp(seed, cursors, lam, width=UNIT_WIDTH, unit0=0):
    lam = _d(lam)
    n = lam.size
    out, t = np.zeros(n), np.zeros(n)
    lib().or_step_exp(seed, unit0, n, width, _p(cursors, _u64p), _p(lam, _dp), _p(out, _dp), _p(t, _dp))
    return out, t


def step_laplace(seed, cursors, mu, b, width=UNIT_WIDTH, unit0=0):
    """Laplace(mu, b) = mu + b (E1 - E2), one E call then another per unit."""
    mu, b = _d(mu), _d(b)
    n = mu.size
    out, t = np.zeros(n), np.zeros(n)
    lib().or_step_laplace(seed, unit0, n, width, _p(cursors, _u64p), _p(mu, _dp), _p(b, _dp),
                          _p(out, _dp), _p(t, _dp))
    return out, t


def step_weibull(seed, cursors, lam, k, width=UNIT_WIDTH, unit0=0):
    """Weibull(lambda, k) = lambda E^(1/k)."""
    lam, k = _d(lam), _d(k)
    n = lam.size
    out, t = np.zeros(n), np.zeros(n)
    lib().or_step_weibull(seed, unit0, n, width, _p(cursors, _u64p), _p(lam, _dp), _p(k, _dp),
                          _p(out, _dp), _p(t, _dp))
    return out, t


def step_gamma(seed, cursors, alpha, width=UNIT_WIDTH, unit0=0):
    """One Gamma(alpha_c, 1) per chain; returns (g, tol, margin, nN, nE)."""
    alpha = _d(alpha)
    n = alpha.size
    out, t, m = np.zeros(n), np.zeros(n), np.zeros(n)
    nN, nE = np.zeros(n, np.int32), np.zeros(n, np.int32)
    lib().or_step_gamma(seed, unit0, n, width, _p(cursors, _u64p), _p(alpha, _dp), _p(out, _dp),
                        _p(t, _dp), _p(m, _dp), _p(nN, _i32p), _p(nE, _i32p))
    return out, t, m, nN, nE


def step_poisson(seed, cursors, lam, width=UNIT_WIDTH, unit0=0):
    """Poisson(lambda) per chain (double precision; U pool): inversion below
    10, Hormann's transformed rejection (PTRS) above; -1 for lambda outside
    [0, 2^30].  Returns (k as int32, decision margin)."""
    lam = _d(lam)
    n = lam.size
    out = np.zeros(n, dtype=np.int32)
    mar = np.zeros(n)
    lib().or_step_poisson(seed, unit0, n, width, _p(cursors, _u64p), _p(lam, _dp), _p(out, _i32p),
                          _p(mar, _dp))
    return out, mar


def step_binomial(seed, cursors, n, p, width=UNIT_WIDTH, unit0=0):
    """Binomial(n, p) per chain (double precision; U pool): with p' =
    min(p, 1 - p), inversion when n p' < 10, Hormann's BTRD otherwise,
    mirrored for p > 1/2; -1 for n < 0 or p outside [0, 1].  Returns (k as
    int32, decision margin)."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    p = _d(p)
    m = n.size
    out = np.zeros(m, dtype=np.int32)
    mar = np.zeros(m)
    lib().or_step_binomial(seed, unit0, m, width, _p(cursors, _u64p), _p(n, _i32p), _p(p, _dp),
                           _p(out, _i32p), _p(mar, _dp))
    return out, mar


def step_multinomial(seed, cursors, offsets, n, weights, width=UNIT_WIDTH, unit0=0):
    """Multinomial(n_i, weights of item i) per item (items are the chains of
    64-item units; components by offsets) by conditional binomials on the U
    pool.  Returns (int32 counts per component, margin per item)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.int32)
    w = _d(weights)
    ni = n.size
    out = np.zeros(int(offsets[-1]), dtype=np.int32)
    mar = np.zeros(ni)
    lib().or_step_multinomial(seed, unit0, ni, width, _p(cursors, _u64p), _p(offsets, _i32p),
                              _p(n, _i32p), _p(w, _dp), _p(out, _i32p), _p(mar, _dp))
    return out, mar


def step_dirichlet(seed, cursors, offsets, alpha, unit0=0):
    """One Dirichlet(alpha_i) per item; item i owns alpha[offsets[i]:offsets[i+1]]."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    alpha = _d(alpha)
    n_items = offsets.size - 1
    out, t = np.zeros(alpha.size), np.zeros(alpha.size)
    m = np.zeros(n_items)
    lib().or_step_dirichlet(seed, unit0, n_items, _p(cursors, _u64p), _p(offsets, _i32p), _p(alpha, _dp),
                            _p(out, _dp), _p(t, _dp), _p(m, _dp))
    return out, t, m


def dirichlet_blocks(seed, cursors, alpha, tb, unit0=0):
    """One Dirichlet(alpha) whose components are drawn in blocks of tb, block
    j from unit unit0 + j (cursors[j], advanced in place), normalised by the
    sum of all gammas.  Returns (theta, tol, margin per block)."""
    alpha = _d(alpha)
    K = alpha.size
    nb = -(-K // tb)
    assert cursors.shape[0] >= nb
    out, t, m = np.zeros(K), np.zeros(K), np.zeros(nb)
    lib().or_dirichlet_blocks(seed, unit0, K, tb, _p(cursors, _u64p), _p(alpha, _dp), _p(out, _dp),
                              _p(t, _dp), _p(m, _dp))
    return out, t, m


def multinomial(seed, cursors, offsets, ntok, theta, unit0=0):
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    ntok = np.ascontiguousarray(ntok, dtype=np.int32)
    theta = _d(theta)
    counts = np.zeros(theta.size, dtype=np.int32)
    lib().or_multinomial(seed, unit0, offsets.size - 1, _p(cursors, _u64p), _p(offsets, _i32p),
                         _p(ntok, _i32p), _p(theta, _dp), _p(counts, _i32p))
    return counts


# --------------------------------------------------------------------------
# Chain models
# --------------------------------------------------------------------------

def triangle(seed, n_chains, iters, x0=None, y0=None, cursors=None, trace=True,
             width=UNIT_WIDTH, unit0=0):
    """Eq. 1 / Fig. 1 triangle Gibbs sampler in FP64; returns dict."""
    nu = _n_units(n_chains, width)
    cur = new_cursors(nu) if cursors is None else cursors
    xf, yf = np.zeros(n_chains), np.zeros(n_chains)
    xtr = np.zeros((iters, n_chains)) if trace else None
    ytr = np.zeros((iters, n_chains)) if trace else None
    x0 = None if x0 is None else _d(x0)
    y0 = None if y0 is None else _d(y0)
    lib().or_triangle(seed, unit0, n_chains, width, iters, _p(x0, _dp), _p(y0, _dp), _p(cur, _u64p),
                      _p(xtr, _dp), _p(ytr, _dp), _p(xf, _dp), _p(yf, _dp))
    return dict(x=xf, y=yf, xtrace=xtr, ytrace=ytr, cursors=cur)


def normexp(seed, n_chains, steps, s0=None, cursors=None, width=UNIT_WIDTH, unit0=0):
    """s' ~ N(0.9 s, 0.5 + |s|), e ~ Exp(1 + s'^2); fresh when s0 is None."""
    nu = _n_units(n_chains, width)
    cur = new_cursors(nu) if cursors is None else cursors
    s = np.zeros(n_chains) if s0 is None else _d(s0).copy()
    str_, etr = np.zeros((steps, n_chains)), np.zeros((steps, n_chains))
    stol, etol = np.zeros((steps, n_chains)), np.zeros((steps, n_chains))
    lib().or_normexp(seed, unit0, n_chains, width, steps, 1 if s0 is None else 0, _p(s, _dp),
                     _p(cur, _u64p), _p(str_, _dp), _p(etr, _dp), _p(stol, _dp), _p(etol, _dp))
    return dict(s=s, strace=str_, etrace=etr, stol=stol, etol=etol, cursors=cur)


def expchain(seed, n_chains, steps, e0=None, cursors=None, width=UNIT_WIDTH, unit0=0):
    """e' ~ Exp(1 + e^2) (rate); fresh (e_0 = first exponential) when e0 is None."""
    nu = _n_units(n_chains, width)
    cur = new_cursors(nu) if cursors is None else cursors
    e = np.zeros(n_chains) if e0 is None else _d(e0).copy()
    etr, etol = np.zeros((steps, n_chains)), np.zeros((steps, n_chains))
    lib().or_expchain(seed, unit0, n_chains, width, steps, 1 if e0 is None else 0, _p(e, _dp),
                      _p(cur, _u64p), _p(etr, _dp), _p(etol, _dp))
    return dict(e=e, etrace=etr, etol=etol, cursors=cur)


def convert(kind: int, w) -> np.ndarray:
    """Entries made from caller-supplied words (pool conversion rules)."""
    w = np.ascontiguousarray(w, dtype=np.uint32)
    out = np.zeros(w.size // 2 if kind == KIND_U64 else w.size, dtype=np.float64)
    lib().or_convert(kind, _p(w, _u32p), w.size, _p(out, _dp))
    return out


def u32_many(w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.uint32)
    out = np.zeros(w.size, dtype=np.float64)
    lib().or_u32_many(_p(w, _u32p), w.size, _p(out, _dp))
    return out


def sort_by_length(steps) -> np.ndarray:
    """Slot order: chains stably sorted by descending step count."""
    steps = np.asarray(steps)
    return np.argsort(-steps.astype(np.int64), kind="stable").astype(np.int32)


def gamma_chain(seed, alpha0, steps, perm=None, cursors=None, width=UNIT_WIDTH, unit0=0):
    """alpha_{t+1} = 0.1 + g_t, g_t ~ Gamma(alpha_t, 1); traces are [t][slot].
    gr0/gr1 are the rounds (per unit, from this call's first) in which each
    draw started and completed, -1 where a chain has no step t."""
    alpha = _d(alpha0).copy()
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    n = alpha.size
    if perm is None:
        perm = sort_by_length(steps)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    nu = _n_units(n, width)
    cur = new_cursors(nu) if cursors is None else cursors
    smax = int(steps.max()) if n else 0
    gtr, gtol, gmar = (np.full((smax, n), np.nan) for _ in range(3))
    gr0, gr1 = (np.full((smax, n), -1, dtype=np.int32) for _ in range(2))
    lib().or_gamma_chain(seed, unit0, n, width, _p(perm, _i32p), _p(steps, _i32p), _p(alpha, _dp),
                         _p(cur, _u64p), _p(gtr, _dp), _p(gtol, _dp), _p(gmar, _dp),
                         _p(gr0, _i32p), _p(gr1, _i32p))
    return dict(alpha=alpha, gtrace=gtr, gtol=gtol, gmargin=gmar, gr0=gr0, gr1=gr1, perm=perm,
                cursors=cur)


# --------------------------------------------------------------------------
# Per-step replay of the fp32 chain models: every output recomputed from the
# state the tested run held before that step (an exact input), so that each
# output is held to the single-result bar instead of a bound propagated along
# the chain.
# --------------------------------------------------------------------------

def normexp_replay(seed, s_in, sp_in, fresh, cursors=None, width=UNIT_WIDTH, unit0=0):
    """s_in[t][c]: state before step t; sp_in[t][c]: the s' the tested run
    used for step t's exponential.  fresh: the starting N call is consumed
    (s0/s0tol report it).  Returns dict with strace/stol/etrace/etol."""
    s_in = _d(s_in)
    sp_in = _d(sp_in)
    steps, n = s_in.shape
    nu = _n_units(n, width)
    cur = new_cursors(nu) if cursors is None else cursors
    s0, s0t = np.zeros(n), np.zeros(n)
    str_, etr, stol, etol = (np.zeros((steps, n)) for _ in range(4))
    lib().or_normexp_replay(seed, unit0, n, width, steps, 1 if fresh else 0, _p(s_in, _dp),
                            _p(sp_in, _dp), _p(cur, _u64p), _p(s0, _dp), _p(s0t, _dp),
                            _p(str_, _dp), _p(etr, _dp), _p(stol, _dp), _p(etol, _dp))
    return dict(s0=s0, s0tol=s0t, strace=str_, stol=stol, etrace=etr, etol=etol, cursors=cur)


def expchain_replay(seed, e_in, fresh, cursors=None, width=UNIT_WIDTH, unit0=0):
    """e_in[t][c]: state before step t.  fresh: the starting E call is
    consumed (e0/e0tol report it)."""
    e_in = _d(e_in)
    steps, n = e_in.shape
    nu = _n_units(n, width)
    cur = new_cursors(nu) if cursors is None else cursors
    e0, e0t = np.zeros(n), np.zeros(n)
    etr, etol = np.zeros((steps, n)), np.zeros((steps, n))
    lib().or_expchain_replay(seed, unit0, n, width, steps, 1 if fresh else 0, _p(e_in, _dp),
                             _p(cur, _u64p), _p(e0, _dp), _p(e0t, _dp), _p(etr, _dp), _p(etol, _dp))
    return dict(e0=e0, e0tol=e0t, etrace=etr, etol=etol, cursors=cur)


def gamma_chain_replay(seed, shape, steps, perm=None, cursors=None, width=UNIT_WIDTH, unit0=0):
    """shape[t][slot]: the shape of each slot's draw at step t (exact).
    steps per chain (user order), perm slot -> chain.  Outputs as
    gamma_chain (traces [t][slot])."""
    shape = _d(shape)
    steps = np.ascontiguousarray(steps, dtype=np.int32)
    smax, n = shape.shape
    if perm is None:
        perm = sort_by_length(steps)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    nu = _n_units(n, width)
    cur = new_cursors(nu) if cursors is None else cursors
    gtr, gtol, gmar = (np.full((smax, n), np.nan) for _ in range(3))
    gr0, gr1 = (np.full((smax, n), -1, dtype=np.int32) for _ in range(2))
    lib().or_gamma_chain_replay(seed, unit0, n, width, _p(perm, _i32p), _p(steps, _i32p),
                                _p(shape, _dp), _p(cur, _u64p), _p(gtr, _dp), _p(gtol, _dp),
                                _p(gmar, _dp), _p(gr0, _i32p), _p(gr1, _i32p))
    return dict(gtrace=gtr, gtol=gtol, gmargin=gmar, gr0=gr0, gr1=gr1, perm=perm, cursors=cur)


def chain_shapes_fp32(alpha0_slots, g):
    """Shapes an fp32 gamma chain forms: row 0 the starting shapes, row t the
    fp32 sum 0.1f + g[t-1] (g: [t][slot] fp32 draws).  Plain fp32 addition,
    correctly rounded, as the chain's definition alpha' = 0.1 + g states it
    in that precision."""
    g32 = np.asarray(g, dtype=np.float32)
    out = np.empty(g32.shape, dtype=np.float32)
    out[0] = np.asarray(alpha0_slots, dtype=np.float32)
    if g32.shape[0] > 1:
        out[1:] = np.float32(0.1) + g32[:-1]
    return out.astype(np.float64)


def lda(seed, offsets, ntok, sweeps, counts0=None, cursors=None, unit0=0):
    """Dirichlet(0.1 + counts) then Multinomial(n_d, theta), per document."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    ntok = np.ascontiguousarray(ntok, dtype=np.int32)
    nd = offsets.size - 1
    total = int(offsets[-1])
    counts = (np.zeros(total, np.int32) if counts0 is None
              else np.ascontiguousarray(counts0, dtype=np.int32).copy())
    cur = new_cursors(nd) if cursors is None else cursors
    thtr, thtol = np.zeros((sweeps, total)), np.zeros((sweeps, total))
    cntr = np.zeros((sweeps, total), np.int32)
    gmar, mmar = np.zeros((sweeps, nd)), np.zeros((sweeps, nd))
    lib().or_lda(seed, unit0, nd, _p(offsets, _i32p), _p(ntok, _i32p), sweeps, _p(counts, _i32p),
                 _p(cur, _u64p), _p(thtr, _dp), _p(thtol, _dp), _p(cntr, _i32p),
                 _p(gmar, _dp), _p(mmar, _dp))
    return dict(counts=counts, theta=thtr, theta_tol=thtol, ctrace=cntr, gmargin=gmar,
                mmargin=mmar, cursors=cur)


# --------------------------------------------------------------------------
# Full LDA: topic-word and document-topic Dirichlets with per-token topics
# (the motivating application of Sec. 1 and its footnote, run as the
# uncollapsed Gibbs sampler of the LDA model: phi_k | z ~ Dir(beta + n_k.),
# theta_d | z ~ Dir(alpha + n_d.), z_di | theta, phi ~ Cat(theta_dk phi_k,w)).
# Units: topic k's vocabulary block j is unit k nb + j (nb blocks of
# LDA_FULL_VBLOCK words per topic), document d is unit K nb + d.
# --------------------------------------------------------------------------

def lda_full_counts(K, V, doc_offsets, words, z):
    """n_dk [D][K] and n_kw [K][V] of an assignment (plain counting; tokens
    with z < 0 or a word outside [0, V) are not counted)."""
    doc_offsets = np.asarray(doc_offsets, dtype=np.int64)
    words = np.asarray(words, dtype=np.int64)
    z = np.asarray(z, dtype=np.int64)
    D = doc_offsets.size - 1
    ndk = np.zeros((D, K), dtype=np.int32)
    nkw = np.zeros((K, V), dtype=np.int32)
    doc = np.repeat(np.arange(D), np.diff(doc_offsets))
    ok = (z >= 0) & (z < K) & (words >= 0) & (words < V)
    np.add.at(ndk, (doc[ok], z[ok]), 1)
    np.add.at(nkw, (z[ok], words[ok]), 1)
    return ndk, nkw


def lda_full_token_topic(theta_d, phi, w, u):
    """One token's topic from the fp32 theta row of its document, the fp32
    topic-word matrix, its word id and its uniform u (a pool entry).  The
    weights p_k = theta_k phi_k,w are formed in fp32 and quantised against
    the binade of their maximum m = f 2^e (f in [1/2, 1)): q_k =
    rint(p_k 2^(24 - e)), an exact scaling, so q of the largest weight is in
    [2^23, 2^24] and the decision is an integer one that both sides take in
    the same precision; with
    C_k = q_0 + ... + q_k, j = (u 2^24 - 1) / 2 and t = (j C_{K-1}) >> 23, the
    topic is the first k with t < C_k (the multinomial rule of the chain
    model, over per-token weights).  A word outside [0, V) gives -1."""
    K, V = phi.shape
    if not (0 <= w < V):
        return -1
    p = np.asarray(theta_d, dtype=np.float32) * np.asarray(phi[:, w], dtype=np.float32)
    m = p.max()
    if m > 0:
        e = int(np.frexp(m)[1])
        q = np.rint(np.ldexp(p, 24 - e)).astype(np.int64)
    else:
        q = np.ones(K, dtype=np.int64)
    c = np.cumsum(q)
    j = (int(round(float(u) * 16777216.0)) - 1) >> 1
    t = (j * int(c[-1])) >> 23
    return int(np.searchsorted(c, t, side="right"))


LDA_FULL_VBLOCK = 1024  # words per topic block: one unit, one gamma stream


def lda_full_units(K, V, D, vblock=LDA_FULL_VBLOCK):
    """Units of a full LDA corpus: topic k's word block j is unit k nb + j
    (nb = ceil(V / vblock) blocks per topic), document d is unit K nb + d."""
    return K * (-(-V // vblock)) + D


def lda_full_sweep(seed, cursors, K, V, alpha, beta, doc_offsets, words, z_in,
                   theta32=None, phi32=None, docs=None, vblock=LDA_FULL_VBLOCK):
    """One sweep from assignment z_in.  Topic k draws phi_k ~ Dir(beta + n_k.)
    with the gammas of words [j vblock, (j + 1) vblock) from unit k nb + j
    (dirichlet_blocks), document d draws theta_d ~ Dir(alpha + n_d.) from
    unit K nb + d, then takes one uniform per token in token order and draws
    the token's topic by lda_full_token_topic.  The shapes beta + n and
    alpha + n are formed in fp32, as the sampler receives them.  The token
    step uses theta32 / phi32 when given (the device's fp32 values, for
    replay), else this sweep's own values rounded to fp32.  cursors
    ([lda_full_units][4], uint64) advance in place.  Returns the fp64 phi and
    theta with their tolerances and decision margins (phi_margin per topic:
    the smallest of its blocks'), the new assignment and its counts.  With
    `docs` (document indices) only those documents draw (every topic still
    does): the other documents' theta rows are NaN, their tokens keep z_in,
    and no counts are returned."""
    doc_offsets = np.ascontiguousarray(doc_offsets, dtype=np.int32)
    words = np.asarray(words, dtype=np.int64)
    D = doc_offsets.size - 1
    nb = -(-V // vblock)
    ndk, nkw = lda_full_counts(K, V, doc_offsets, words, z_in)
    a_phi = (np.float32(beta) + nkw.astype(np.float32)).astype(np.float32)
    a_th = (np.float32(alpha) + ndk.astype(np.float32)).astype(np.float32).ravel()
    off_th = (np.arange(D + 1, dtype=np.int32) * K).astype(np.int32)
    phi, phi_t, phi_m = np.zeros((K, V)), np.zeros((K, V)), np.zeros(K)
    for k in range(K):
        ck = cursors[k * nb:(k + 1) * nb]  # a view: advanced in place
        phi[k], phi_t[k], mb = dirichlet_blocks(seed, ck, a_phi[k], vblock, unit0=k * nb)
        phi_m[k] = mb.min()
    cd = cursors[K * nb:]
    du = K * nb  # unit of document 0
    if docs is None:
        th, th_t, th_m = step_dirichlet(seed, cd, off_th, a_th, unit0=du)
        todo = range(D)
    else:
        th, th_t, th_m = np.full(D * K, np.nan), np.full(D * K, np.nan), np.full(D, np.nan)
        for d in docs:
            c1 = cd[d:d + 1]  # this document's cursors, advanced in place
            o1 = np.array([0, K], dtype=np.int32)
            r1 = step_dirichlet(seed, c1, o1, a_th[d * K:(d + 1) * K], unit0=du + int(d))
            th[d * K:(d + 1) * K], th_t[d * K:(d + 1) * K], th_m[d] = r1[0], r1[1], r1[2][0]
        todo = docs
    phi_f = (phi.astype(np.float32) if phi32 is None else np.asarray(phi32, np.float32)).reshape(K, V)
    th_f = (th.astype(np.float32) if theta32 is None else np.asarray(theta32, np.float32)).reshape(D, K)
    z = (np.full(words.size, -1, dtype=np.int32) if docs is None
         else np.asarray(z_in, dtype=np.int32).copy())
    for d in todo:
        a, b = int(doc_offsets[d]), int(doc_offsets[d + 1])
        if b == a:
            continue
        u = entries(seed, du + d, KIND_U, int(cd[d, KIND_U]), b - a)
        cd[d, KIND_U] += np.uint64(b - a)
        for i in range(a, b):
            z[i] = lda_full_token_topic(th_f[d], phi_f, int(words[i]), u[i - a])
    ndk2, nkw2 = lda_full_counts(K, V, doc_offsets, words, z) if docs is None else (None, None)
    return dict(phi=phi.reshape(K, V), phi_tol=phi_t.reshape(K, V), phi_margin=phi_m,
                theta=th.reshape(D, K), theta_tol=th_t.reshape(D, K), theta_margin=th_m,
                z=z, ndk=ndk2, nkw=nkw2, cursors=cursors)
