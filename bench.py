#!/usr/bin/env python3
"""Benchmark of the varying-parameter pool RNG on one MI355X.

Headline workload (LDA-style Dirichlet resampling): 16,384 documents with
K uniform on {8, 16, 64, 256} components and Poisson(200) tokens, 100 sweeps
per step; each sweep draws theta ~ Dirichlet(0.1 + counts) from K gammas and
then counts ~ Multinomial(n, theta) from the document's uniforms.  fp32
deviates, int32 counts, Philox4x32-10 pools of an autotuned window per
document per kind, regenerated in place when they run out.  One timed step
is the whole hot path over that batch: bulk refill of the pool windows (one
128-bit store per Philox block) followed by one launch that runs every
document for all its sweeps, writing theta and the counts of every sweep.
Documents continue from step to step.

After it, under "workloads": the varying-shape gamma chains (262,144 chains
of uneven length 50..1,000 with alpha_{t+1} = 0.1 + g_t) and the
normal/exponential chains (65,536 chains x 1,000 steps, s' ~ N(0.9 s,
0.5 + |s|) then e ~ Exp(1 + s'^2)), measured the same way (a step refills
only the windows its chain kernel reads: none for the gamma chains, whose
kernel generates every entry it consumes).  --workload runs
one workload alone: triangle (Eq. 1 / Fig. 1, 1,024 chains x 10,000
iterations, fp64), normexp, gamma, lda, lda_full (full LDA on a synthetic
corpus: 16,384 documents, 64 topics (--lda-topics), 4,096 words
(--lda-vocab), per sweep the topic-word
and document-topic Dirichlets and one topic per token), served (the mixed
request stream alone).

Prints one JSON line: deviates/s, the roofline of the dominant kernel
(algorithmic bytes over its duration against 8 TB/s; the duration from HIP
events that the launch itself records at the kernel's start and end, with
the span of the call on the stream beside it), the CPU oracle timed on the
host over a stated sample (all worker processes, and one thread with its
cycles per deviate at the host's nominal clock; CPU model, logical CPUs,
sockets and clock recorded), and (unless --no-served) the served form
against per-request plain launches on a mixed request stream at the full
size ranges (chains log-U[1, 65,536], steps log-U[10, 10,000]): throughput
with every request queued, and p50/p99 latency under Poisson arrivals at 70%
of the plain capacity.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_sources_sha() -> str:
    """Digest of the HIP sources and the C header (names and contents)."""
    import glob
    import hashlib
    h = hashlib.sha1()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_1412_4825_amd", "csrc", "*")))
    for f in files + [os.path.join(ROOT, "include", "brng.h")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(label: str):
    """HBM bytes per launch of kernel `label` (FETCH_SIZE + WRITE_SIZE, scaled
    by a known-size copy) from the committed rocprof summaries under
    profiles/, or None when the kernel sources have changed since."""
    import glob
    sha = kernel_sources_sha()
    for p in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(p) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 5 and f[0] == "traffic" and f[1] == label:
                    kv = dict(x.split("=", 1) for x in f[2:])
                    if kv.get("sources") == sha:
                        return float(kv["fetch_bytes"]) + float(kv["write_bytes"])
    return None


class Events:
    """HIP events recorded on the library's stream (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def span(self, name):
        t = self.torch
        a = t.cuda.Event(enable_timing=True)
        b = t.cuda.Event(enable_timing=True)
        a.record()
        self.pairs.setdefault(name, []).append((a, b))
        return b

    def ms(self, name):
        return [a.elapsed_time(b) for a, b in self.pairs.get(name, [])]


def _slices(units, workers):
    per = (units + workers - 1) // workers
    return [(w * per, min(units, (w + 1) * per)) for w in range(workers) if w * per < units]


def _pool_run(fn, jobs):
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        busy = pool.map(fn, jobs)
    return time.perf_counter() - t0, sum(busy)


# ---------------------------------------------------------------------------
# CPU oracle legs (test infrastructure; timed on the host cores)
# ---------------------------------------------------------------------------

def _cpu_normexp(a):
    seed, u0, n, steps = a
    import oracle
    t = time.perf_counter()
    oracle.normexp(seed, n, steps, unit0=u0)
    return time.perf_counter() - t


def _cpu_triangle(a):
    seed, u0, n, iters = a
    import oracle
    t = time.perf_counter()
    oracle.triangle(seed, n, iters, unit0=u0, trace=False)
    return time.perf_counter() - t


def _cpu_gamma(a):
    seed, u0, alpha0, steps = a
    import oracle
    t = time.perf_counter()
    oracle.gamma_chain(seed, alpha0, steps, perm=np.arange(alpha0.size, dtype=np.int32),
                       unit0=u0)
    return time.perf_counter() - t


def _cpu_lda(a):
    seed, d0, offsets, ntok, sweeps = a
    import oracle
    t = time.perf_counter()
    oracle.lda(seed, offsets, ntok, sweeps, unit0=d0)
    return time.perf_counter() - t


# ---------------------------------------------------------------------------
# workloads: each returns the context, the fresh and resume requests, the
# kinds it draws, entry sizes, windows, deviates and output bytes per step,
# its description and the CPU leg
# ---------------------------------------------------------------------------

def setup_normexp(torch, b, args):
    n, steps = args.chains or 65536, args.chain_steps or 1000
    W = args.window or 4096
    dev = torch.device("cuda:0")
    ctx = b.brng_create(args.seed, n, [0, W, W, 0], stream=torch.cuda.current_stream())
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.empty((steps, n), dtype=torch.float32, device=dev)
    te = torch.empty((steps, n), dtype=torch.float32, device=dev)
    kw = dict(max_steps=steps, seed=args.seed, trace=ts, trace2=te, trace_stride=n)
    fresh = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, **kw)
    resume = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, flags=b.BRNG_FLAG_RESUME, **kw)
    units = (n + 63) // 64

    def cpu(workers):
        jobs = [(args.seed, u0, min(n, u1 * 64) - u0 * 64, steps) for u0, u1 in _slices(units, workers)]
        wall, busy = _pool_run(_cpu_normexp, jobs)
        dv = 2 * n * steps
        return {"value": dv / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
                "sample": "whole workload (%d chains x %d steps, %.3g deviates) split by unit "
                          "over %d processes; %.1f s of CPU work" % (n, steps, dv, len(jobs), busy)}

    def cpu1():
        nu = min(units, 16)
        busy = _cpu_normexp((args.seed, 0, min(n, 64 * nu), steps))
        dv = 2 * min(n, 64 * nu) * steps
        return {"value": dv / busy, "unit": "deviates/s", "threads": 1,
                "sample": "the first %d units (%d chains x %d steps) in one thread" % (nu, min(n, 64 * nu), steps)}

    # `keep` holds the device arrays the descriptors point to for as long as
    # the descriptors are used
    return dict(ctx=ctx, fresh=fresh, resume=resume, kinds=[b.BRNG_N, b.BRNG_E], keep=(st, ts, te),
                entry_bytes={b.BRNG_N: 4, b.BRNG_E: 4}, windows={b.BRNG_N: W, b.BRNG_E: W},
                deviates=2 * n * steps, out_bytes=2 * n * steps * 4, dtype="f32", cpu=cpu,
                cpu1=cpu1, kernel="k_gibbs<1>",
                config={"workload": "normal/exponential chains: s'~N(0.9s,0.5+|s|), e~Exp(1+s'^2)",
                        "chains": n, "steps": steps, "window_per_unit_per_kind": W,
                        "unit_chains": 64, "precision": "fp32", "generator": "Philox4x32-10"})


def setup_triangle(torch, b, args):
    n, iters = args.chains or 1024, args.chain_steps or 10000
    W = args.window or 4096
    dev = torch.device("cuda:0")
    ctx = b.brng_create(args.seed, n, [0, 0, 0, W], stream=torch.cuda.current_stream())
    st = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    tx = torch.empty((iters, n), dtype=torch.float64, device=dev)
    ty = torch.empty((iters, n), dtype=torch.float64, device=dev)
    kw = dict(max_steps=iters, seed=args.seed, trace=tx, trace2=ty, trace_stride=n)
    fresh = b.gibbs_desc(b.BRNG_MODEL_TRIANGLE_F64, n, st, **kw)
    resume = b.gibbs_desc(b.BRNG_MODEL_TRIANGLE_F64, n, st, flags=b.BRNG_FLAG_RESUME, **kw)
    units = (n + 63) // 64

    def cpu(workers):
        jobs = [(args.seed, u0, min(n, u1 * 64) - u0 * 64, iters) for u0, u1 in _slices(units, workers)]
        wall, busy = _pool_run(_cpu_triangle, jobs)
        dv = 2 * n * iters
        return {"value": dv / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
                "sample": "whole workload (%d chains x %d iterations) split by unit over %d "
                          "processes; %.1f s of CPU work" % (n, iters, len(jobs), busy)}

    def cpu1():
        nu = min(units, 4)
        m = min(n, 64 * nu)
        busy = _cpu_triangle((args.seed, 0, m, iters))
        return {"value": 2 * m * iters / busy, "unit": "deviates/s", "threads": 1,
                "sample": "the first %d units (%d chains x %d iterations) in one thread" % (nu, m, iters)}

    return dict(ctx=ctx, fresh=fresh, resume=resume, kinds=[b.BRNG_U64], keep=(st, tx, ty),
                entry_bytes={b.BRNG_U64: 8}, windows={b.BRNG_U64: W},
                deviates=2 * n * iters, out_bytes=2 * n * iters * 8, dtype="f64", cpu=cpu, cpu1=cpu1,
                kernel="k_gibbs<0>",
                config={"workload": "triangle Gibbs sampler of Eq. 1 / Fig. 1: x~U(0,1-y), y~U(0,1-x)",
                        "chains": n, "iterations": iters, "window_per_unit": W,
                        "precision": "fp64", "generator": "Philox4x32-10"})


def setup_gamma(torch, b, args):
    from paper_1412_4825_amd import workloads
    n = args.chains or 262144
    wl = workloads.gamma_chain(n_chains=n, seed=args.seed)
    W = args.window or 4096
    dev = torch.device("cuda:0")
    ctx = b.brng_create(args.seed, n, [0, W, W, 0], stream=torch.cuda.current_stream())
    perm = b.brng_sort_by_length(wl["steps"])
    smax = int(wl["steps"].max())
    st = torch.from_numpy(wl["alpha0"]).to(dev)
    tg = torch.empty((smax, n), dtype=torch.float32, device=dev)
    tsteps = torch.from_numpy(wl["steps"]).to(dev)
    tperm = torch.from_numpy(perm).to(dev)
    kw = dict(max_steps=smax, seed=args.seed, trace=tg, trace_stride=n, steps=tsteps, perm=tperm)
    fresh = b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st, **kw)
    resume = b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st, flags=b.BRNG_FLAG_RESUME, **kw)
    draws = int(wl["steps"].sum())
    units = (n + 63) // 64

    def cpu(workers):
        # a sample: the first units of the length-sorted slot order
        su = min(units, args.cpu_units or 1024)
        jobs = []
        for u0, u1 in _slices(su, workers):
            sl = perm[u0 * 64:min(n, u1 * 64)]
            jobs.append((args.seed, u0, wl["alpha0"][sl].astype(np.float64), wl["steps"][sl]))
        wall, busy = _pool_run(_cpu_gamma, jobs)
        dv = int(wl["steps"][perm[:su * 64]].sum())
        return {"value": dv / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
                "sample": "%d of %d units (the longest chains first, %.3g gamma draws) over %d "
                          "processes; %.1f s of CPU work" % (su, units, dv, len(jobs), busy)}

    def cpu1():
        nu = min(units, 16)
        sl = perm[:min(n, 64 * nu)]
        busy = _cpu_gamma((args.seed, 0, wl["alpha0"][sl].astype(np.float64), wl["steps"][sl]))
        dv = int(wl["steps"][sl].sum())
        return {"value": dv / busy, "unit": "deviates/s", "threads": 1,
                "sample": "the first %d units (the longest chains, %d gamma draws) in one thread" % (nu, dv)}

    def oaat(events):
        """The same shapes drawn with one launch per step (brng_step_gamma)."""
        c2 = b.brng_create(args.seed + 1, n, [0, W, W, 0], stream=torch.cuda.current_stream())
        a = torch.from_numpy(wl["alpha0"][perm]).to(dev)
        out = torch.empty(n, dtype=torch.float32, device=dev)
        k = args.oaat_steps
        for _ in range(3):
            b.brng_step_gamma(c2, a, out)
        torch.cuda.synchronize()
        e0 = events.span("oaat")
        for _ in range(k):
            b.brng_step_gamma(c2, a, out)
            torch.add(out, 0.1, out=a)
        e0.record()
        torch.cuda.synchronize()
        b.brng_destroy(c2)
        ms = events.ms("oaat")[0]
        return {"value": n * k / (ms / 1e3), "unit": "deviates/s", "launches": 2 * k,
                "note": "one brng_step_gamma launch per step over all %d chains, alpha update "
                        "on the stream between launches" % n}

    # the chain kernel generates every entry it consumes (its readers never
    # load a window), so no bulk refill precedes it; all pool bytes count
    # as the kernel's
    return dict(ctx=ctx, fresh=fresh, resume=resume, kinds=[b.BRNG_N, b.BRNG_E],
                fill_kinds=[],
                keep=(st, tg, tsteps, tperm),
                entry_bytes={b.BRNG_N: 4, b.BRNG_E: 4}, windows={b.BRNG_N: W, b.BRNG_E: W},
                deviates=draws, out_bytes=draws * 4, dtype="f32", cpu=cpu, cpu1=cpu1, oaat=oaat,
                kernel="k_gibbs<2>",
                config={"workload": "varying-shape gamma chains: g~Gamma(alpha,1), alpha'=0.1+g, "
                                    "Marsaglia-Tsang with the alpha<1 boost",
                        "chains": n, "steps": "U{50..1000}", "draws_per_step": draws,
                        "window_per_unit_per_kind": W, "precision": "fp32",
                        "generator": "Philox4x32-10"})


def setup_lda(torch, b, args):
    from paper_1412_4825_amd import workloads
    nd = args.chains or 16384
    sweeps = args.chain_steps or 100
    wl = workloads.lda(n_docs=nd, sweeps=sweeps, seed=args.seed)
    W = args.window or 4096
    dev = torch.device("cuda:0")
    ctx = b.brng_create(args.seed, nd, [W, W, W, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    total = int(wl["offsets"][-1])
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    th = torch.empty((sweeps, total), dtype=torch.float32, device=dev)
    ct = torch.empty((sweeps, total), dtype=torch.int32, device=dev)
    toff = torch.from_numpy(wl["offsets"]).to(dev)
    tntok = torch.from_numpy(wl["ntok"]).to(dev)
    kw = dict(max_steps=sweeps, seed=args.seed, trace=th, trace2=ct, trace_stride=total,
              offsets=toff, ntok=tntok)
    fresh = b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts, **kw)
    resume = b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts, flags=b.BRNG_FLAG_RESUME, **kw)
    dv = sweeps * (total + int(wl["ntok"].sum()))

    def cpu(workers):
        sd = min(nd, args.cpu_units or 2048)
        jobs = []
        for d0, d1 in _slices(sd, workers):
            off = wl["offsets"][d0:d1 + 1] - wl["offsets"][d0]
            jobs.append((args.seed, d0, off.astype(np.int32), wl["ntok"][d0:d1], sweeps))
        wall, busy = _pool_run(_cpu_lda, jobs)
        sdv = sweeps * (int(wl["offsets"][sd]) + int(wl["ntok"][:sd].sum()))
        return {"value": sdv / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
                "sample": "%d of %d documents x %d sweeps (%.3g deviates) over %d processes; "
                          "%.1f s of CPU work" % (sd, nd, sweeps, sdv, len(jobs), busy)}

    def cpu1():
        sd = min(nd, 64)
        off = wl["offsets"][:sd + 1].astype(np.int32)
        busy = _cpu_lda((args.seed, 0, off, wl["ntok"][:sd], sweeps))
        sdv = sweeps * (int(off[-1]) + int(wl["ntok"][:sd].sum()))
        return {"value": sdv / busy, "unit": "deviates/s", "threads": 1,
                "sample": "the first %d documents x %d sweeps (%.3g deviates) in one thread" % (sd, sweeps, sdv)}

    # the kernel draws the multinomial's uniforms in registers (its U window
    # is never read), so the bulk refill covers N and E; the U entries still
    # count in the algorithmic bytes (a pool round trip each)
    return dict(ctx=ctx, fresh=fresh, resume=resume, kinds=[b.BRNG_U, b.BRNG_N, b.BRNG_E],
                fill_kinds=[b.BRNG_N, b.BRNG_E],
                keep=(counts, th, ct, toff, tntok),
                entry_bytes={b.BRNG_U: 4, b.BRNG_N: 4, b.BRNG_E: 4},
                windows={b.BRNG_U: W, b.BRNG_N: W, b.BRNG_E: W},
                deviates=dv, out_bytes=sweeps * total * 8, dtype="f32", cpu=cpu, cpu1=cpu1,
                kernel="k_gibbs_lda",
                config={"workload": "LDA-style Dirichlet resampling: theta~Dir(0.1+counts), "
                                    "counts~Mult(n_d, theta)",
                        "documents": nd, "sweeps": sweeps, "K": "{8,16,64,256}",
                        "tokens": "Poisson(200)", "components": total,
                        "window_per_unit_per_kind": W, "precision": "fp32 deviates, int32 counts",
                        "generator": "Philox4x32-10"})


def _cpu_lda_full(a):
    seed, K, V, off, words, z0, alpha, beta, docs = a
    import oracle
    t = time.perf_counter()
    cur = oracle.new_cursors(oracle.lda_full_units(K, V, off.size - 1))
    oracle.lda_full_sweep(seed, cur, K, V, alpha, beta, off, words, z0, docs=docs)
    return time.perf_counter() - t


def setup_lda_full(torch, b, args):
    """Full LDA on a synthetic corpus: per sweep K topic-word Dirichlets over
    the vocabulary, one document-topic Dirichlet per document and one topic
    per token.  A step is one call of `sweeps_per_step` sweeps."""
    from paper_1412_4825_amd import workloads
    nd = args.chains or 16384
    K, V = args.lda_topics, args.lda_vocab
    sweeps = args.chain_steps or 5
    alpha, beta = 0.1, 0.05
    c = workloads.lda_corpus(n_docs=nd, n_topics=K, n_vocab=V, seed=args.seed)
    T = int(c["offsets"][-1])
    W = args.window or 512
    dev = torch.device("cuda:0")
    n_units = b.brng_lda_full_units(K, V, nd)
    du = n_units - nd  # topic-block units first, then one unit per document
    ctx = b.brng_create(args.seed, n_units, [W, W, W, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    toff = torch.from_numpy(c["offsets"]).to(dev)
    tw = torch.from_numpy(c["words"]).to(dev)
    tz = torch.from_numpy(c["z0"]).to(dev)
    ndk = torch.zeros(nd * K, dtype=torch.int32, device=dev)
    nkw = torch.zeros(K * V, dtype=torch.int32, device=dev)
    th = torch.zeros(nd * K, dtype=torch.float32, device=dev)
    phi = torch.zeros(K * V, dtype=torch.float32, device=dev)

    state = {"counted": False}

    def run():
        # the first call counts the starting assignment; later calls get the
        # counts the previous call returned
        b.brng_run_lda_full(ctx, K, V, sweeps, alpha, beta, toff, tw, tz, ndk, nkw, th, phi,
                            counts_valid=state["counted"])
        state["counted"] = True

    dv = sweeps * (K * V + nd * K + T)
    # outputs per sweep: phi, theta, z, n_dk, n_kw, and the corpus's words read
    out_b = sweeps * 4.0 * (2 * K * V + 2 * nd * K + 2 * T)

    def kernel_bytes(delta):
        # the document kernel of one sweep: its units' consumed entries (the
        # document units), written once and read once, plus theta, z,
        # n_d., the n_kw increments and the words it reads
        ent = delta[du:, [b.BRNG_U, b.BRNG_N, b.BRNG_E]].sum() / sweeps
        return 8.0 * ent + 4.0 * (2 * nd * K + 3 * T)

    def cpu(workers):
        # one sweep over the first sd documents, the documents split over the
        # workers (each also draws the topics, counted once)
        sd = min(nd, args.cpu_units or 4096)
        off = c["offsets"][:sd + 1].astype(np.int32)
        n = int(off[-1])
        jobs = [(args.seed, K, V, off, c["words"][:n], c["z0"][:n], alpha, beta,
                 list(range(d0, d1))) for d0, d1 in _slices(sd, workers)]
        wall, busy = _pool_run(_cpu_lda_full, jobs)
        sdv = K * V + sd * K + n
        return {"value": sdv / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
                "sample": "one sweep of the first %d of %d documents (%d x %d topic-word draws, "
                          "%d tokens; %.3g deviates) over %d processes, each drawing the topics "
                          "and its documents; %.1f s of CPU work"
                          % (sd, nd, K, V, n, sdv, len(jobs), busy)}

    def cpu1():
        sd = min(nd, 256)
        off = c["offsets"][:sd + 1].astype(np.int32)
        n = int(off[-1])
        busy = _cpu_lda_full((args.seed, K, V, off, c["words"][:n], c["z0"][:n], alpha, beta,
                              list(range(sd))))
        sdv = K * V + sd * K + n
        return {"value": sdv / busy, "unit": "deviates/s", "threads": 1,
                "sample": "one sweep of the topics and the first %d documents (%.3g deviates) "
                          "in one thread" % (sd, sdv)}

    return dict(ctx=ctx, run=run, kinds=[b.BRNG_U, b.BRNG_N, b.BRNG_E],
                keep=(toff, tw, tz, ndk, nkw, th, phi),
                entry_bytes={b.BRNG_U: 4, b.BRNG_N: 4, b.BRNG_E: 4},
                windows={b.BRNG_U: W, b.BRNG_N: W, b.BRNG_E: W},
                deviates=dv, out_bytes=out_b, dtype="f32", cpu=cpu, cpu1=cpu1,
                kernel="k_ldaf_docs", kernel_bytes=kernel_bytes,
                config={"workload": "full LDA, uncollapsed Gibbs on a synthetic corpus: "
                                    "phi_k~Dir(beta+n_k.), theta_d~Dir(alpha+n_d.), "
                                    "z~Cat(theta_d phi_.w)",
                        "documents": nd, "topics": K, "vocabulary": V, "tokens": T,
                        "tokens_per_document": "Poisson(200)", "alpha": alpha, "beta": beta,
                        "sweeps_per_step": sweeps, "window_per_unit_per_kind": W,
                        "precision": "fp32 deviates, int32 topics and counts",
                        "generator": "Philox4x32-10"})


def copy_bandwidth(torch, b, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth for context: the library's streaming
    conversion kernel (brng_convert, uniform kind: one 16-byte load and one
    16-byte store per thread) over `nbytes` of words, read + write bytes over
    event time."""
    n = nbytes // 4
    src = torch.randint(0, 2 ** 31 - 1, (n,), dtype=torch.int32, device="cuda")
    dst = torch.empty(n, dtype=torch.float32, device="cuda")
    b.brng_convert(b.BRNG_U, src, n, dst, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.brng_convert(b.BRNG_U, src, n, dst, stream=torch.cuda.current_stream())
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    return gbs


def per_distribution(torch, b, args, n=1 << 20, calls=20):
    """The paper's results table on one MI355X, per distribution (Sec. 2.4):
    the bulk fill of a pool (its Batch column) and one-at-a-time calls with a
    different parameter per chain and per call (its BatchRNG column; each
    call is one launch over n chains), in deviates/s."""
    from paper_1412_4825_amd import workloads
    dev = torch.device("cuda:0")
    W = 4096
    p = workloads.step_params(n, seed=args.seed)
    t = {k: torch.from_numpy(v).to(dev) for k, v in p.items()}
    shape = torch.from_numpy(np.exp(np.random.default_rng(1).uniform(
        np.log(0.2), np.log(20.0), n)).astype(np.float32)).to(dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    ctx = b.brng_create(args.seed, n, [W, W, W, 0], stream=torch.cuda.current_stream())
    res = {}
    try:
        def timed(fn, count):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(calls):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return count * calls / (e0.elapsed_time(e1) / 1e3)

        units = (n + 63) // 64
        for name, kind in (("uniform", b.BRNG_U), ("normal", b.BRNG_N), ("exponential", b.BRNG_E)):
            res[name] = {"batch_fill": timed(lambda: b.brng_fill_base(ctx, kind), units * W)}
        res["uniform"]["one_at_a_time"] = timed(lambda: b.brng_step_uniform(ctx, t["a"], t["b"], out), n)
        res["normal"]["one_at_a_time"] = timed(lambda: b.brng_step_normal(ctx, t["mu"], t["sigma"], out), n)
        res["exponential"]["one_at_a_time"] = timed(lambda: b.brng_step_exp(ctx, t["lam"], out), n)
        res["laplace"] = {"one_at_a_time": timed(lambda: b.brng_step_laplace(ctx, t["mu"], t["sigma"], out), n)}
        res["weibull"] = {"one_at_a_time": timed(lambda: b.brng_step_weibull(ctx, t["lam"], shape, out), n)}
        res["gamma"] = {"one_at_a_time": timed(lambda: b.brng_step_gamma(ctx, t["alpha"], out), n)}
        # Poisson rates log-uniform in [0.1, 1000]: both the inversion and
        # the transformed-rejection path
        rate = torch.from_numpy(np.exp(np.random.default_rng(2).uniform(
            np.log(0.1), np.log(1000.0), n)).astype(np.float32)).to(dev)
        kout = torch.empty(n, dtype=torch.int32, device=dev)
        res["poisson"] = {"one_at_a_time": timed(lambda: b.brng_step_poisson(ctx, rate, kout), n)}
        # binomial: n log-uniform in [1, 10^4], p uniform: both paths
        g2 = np.random.default_rng(3)
        trials = torch.from_numpy(np.floor(np.exp(g2.uniform(0, np.log(1e4), n))).astype(np.int32)).to(dev)
        prob = torch.from_numpy(g2.uniform(size=n).astype(np.float32)).to(dev)
        res["binomial"] = {"one_at_a_time": timed(lambda: b.brng_step_binomial(ctx, trials, prob, kout), n)}
        # multinomial by conditional binomials: 8 components per item, the
        # same trial counts; deviates = items x components
        moff = torch.arange(0, 8 * n + 1, 8, dtype=torch.int32, device=dev)
        mw = torch.from_numpy(g2.exponential(size=8 * n).astype(np.float32)).to(dev)
        mout = torch.empty(8 * n, dtype=torch.int32, device=dev)
        res["multinomial_k8"] = {"one_at_a_time": timed(
            lambda: b.brng_step_multinomial(ctx, moff, trials, mw, mout), 8 * n)}
    finally:
        b.brng_destroy(ctx)
    return {"chains": n, "calls": calls, "window": W, "unit": "deviates/s",
            "rates": {k: {c: float("%.4g" % v) for c, v in d.items()} for k, d in res.items()}}


def autotune_launch(torch, b, args):
    """Pick the pool window and waves per workgroup for the gamma/LDA
    workloads by timing one step (bulk refills + the resumed chain launch)
    per candidate (results do not depend on either)."""
    import copy

    from paper_1412_4825_amd import autotune
    setup = WORKLOADS[args.workload]

    def trial_factory():
        cache = {}

        def trial(window, wpb):
            if window not in cache:
                for old in cache.values():
                    b.brng_destroy(old["ctx"])
                cache.clear()
                a2 = copy.copy(args)
                a2.window = window
                Wk = setup(torch, b, a2)
                b.brng_run_gibbs(Wk["ctx"], Wk["fresh"])
                cache[window] = Wk
            Wk = cache[window]
            b.brng_set_launch(Wk["ctx"], wpb)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()  # one whole step: the bulk refills and the chain launch
            for k in Wk.get("fill_kinds", Wk["kinds"]):
                b.brng_fill_base(Wk["ctx"], k)
            b.brng_run_gibbs(Wk["ctx"], Wk["resume"])
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / 1e3

        return trial, cache

    trial, cache = trial_factory()
    best = autotune.pick(trial, windows=(512, 1024, 2048, 4096), wpbs=(2, 4, 8), reps=2)
    for Wk in cache.values():
        b.brng_destroy(Wk["ctx"])
    torch.cuda.synchronize()
    return best


def served_section(torch, args, n_req):
    """The served form against per-request plain launches on the same mixed
    request stream: capacity (all requests queued at once) and latency
    (Poisson arrivals at 70% of the plain capacity, measured on a
    500-request prefix)."""
    from paper_1412_4825_amd import serve, workloads
    dev = torch.device("cuda:0")
    qs = workloads.served_requests(n_req, chains_max=args.served_chains_max,
                                   steps_max=args.served_steps_max, seed=args.seed)
    # every request returns its final state and per-chain sums of its outputs
    reqs = [serve.Request(torch, q, dev, sums=True) for q in qs]
    W = [4096] * 4
    deviates = sum(r.deviates for r in reqs)
    for r in reqs:
        r.reset()

    def say(*a):
        print("[served]", *a, file=sys.stderr, flush=True)

    # plain launches in chunks of 100 requests (one context per chunk), with
    # a progress line per chunk
    service = []
    for i in range(0, n_req, 100):
        service.append(serve.run_plain(torch, reqs[i:i + 100], W))
        say("plain", min(i + 100, n_req), "of", n_req)
    service = np.concatenate(service)
    k = min(500, n_req)
    mu_p = k / service[:k].sum()
    rate = 0.7 * mu_p
    arrivals = workloads.poisson_arrivals(n_req, rate, seed=args.seed)
    lat_plain = serve.fifo_latency(arrivals, service)
    kw = dict(budget=args.served_budget_mb << 20, window=W, max_active=args.served_slots,
              tick_steps=args.served_tick_steps, tick_sweeps=args.served_tick_sweeps,
              max_bypass_ms=args.served_bypass_ms)
    kw["on_done"] = lambda d: say("served", d, "of", n_req) if d % 100 == 0 else None
    for r in reqs:
        r.reset()
    _, makespan, st_sat = serve.run_served(torch, reqs, np.zeros(n_req), **kw)
    for r in reqs:
        r.reset()
    lat_srv, span_srv, st = serve.run_served(torch, reqs, arrivals, **kw)

    def pct(x):
        return {"p50_ms": round(float(np.percentile(x, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(x, 99)) * 1e3, 3)}

    kinds = {kd: sum(1 for q in qs if q["kind"] == kd) for kd in workloads.SERVED_KINDS}
    return {
        "requests": n_req, "kinds": kinds, "deviates": deviates,
        "served": dict(capacity_deviates_per_s=deviates / makespan,
                       makespan_s=round(makespan, 4), ticks=st_sat["ticks"],
                       peak_bytes=st_sat["bytes_peak"], **pct(lat_srv)),
        "plain": dict(capacity_deviates_per_s=deviates / service.sum(),
                      busy_s=round(float(service.sum()), 4), **pct(lat_plain)),
        "arrival_rate_per_s": round(rate, 2), "load": "0.7 x plain capacity (first %d requests)" % k,
        "chains": "log-U[1, %d]" % args.served_chains_max,
        "steps": "log-U[10, %d]" % args.served_steps_max,
        "server": dict(budget_mb=args.served_budget_mb, slots=args.served_slots,
                       tick_steps=args.served_tick_steps, tick_sweeps=args.served_tick_sweeps,
                       max_bypass_ms=args.served_bypass_ms, window=W[0]),
        "outputs": "final state + per-chain sum and sum of squares of every output",
    }


def served_main(torch, args):
    t0 = time.perf_counter()
    sec = served_section(torch, args, args.served_requests)
    out = {
        "metric": "served p50/p99 latency vs plain; deviates/s",
        "value": sec["served"]["capacity_deviates_per_s"],
        "unit": "deviates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": sec["served"]["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "served mixed request stream (uniform/normal/exponential/gamma/"
                               "Dirichlet chains), continuous batching vs per-request plain "
                               "launches", "requests": sec["requests"], "chains": sec["chains"],
                   "steps": sec["steps"]},
        "roofline": None,
        "cpu_baseline": None,
        "served": sec,
        "wall_s": round(time.perf_counter() - t0, 2),
    }
    print(json.dumps(out), flush=True)


WORKLOADS = {"normexp": setup_normexp, "triangle": setup_triangle, "gamma": setup_gamma,
             "lda": setup_lda, "lda_full": setup_lda_full}


def host_cpu_info():
    """The host's CPU model, logical CPUs, sockets and nominal clock (GHz), as
    the system reports them; fields it does not report are None."""
    info = {"cpu_model": None, "nproc": os.cpu_count(), "sockets": None, "nominal_ghz": None,
            "nominal_ghz_source": None}
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in txt.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["cpu_model"] = kv.get("Model name")
        if kv.get("Socket(s)", "").isdigit():
            info["sockets"] = int(kv["Socket(s)"])
        if "CPU max MHz" in kv:
            info["max_ghz"] = round(float(kv["CPU max MHz"]) / 1e3, 3)
    except Exception:
        pass
    try:
        info["nproc"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    # nominal (base) clock: the cpufreq driver's nominal or base frequency
    # (kHz), else a frequency printed in the model name
    for f in ("amd_pstate_nominal_freq", "base_frequency"):
        path = "/sys/devices/system/cpu/cpu0/cpufreq/" + f
        try:
            with open(path) as fh:
                info["nominal_ghz"] = round(int(fh.read().strip()) / 1e6, 3)
                info["nominal_ghz_source"] = path
                break
        except Exception:
            continue
    if info["nominal_ghz"] is None and info["cpu_model"] and "GHz" in info["cpu_model"]:
        import re
        m = re.search(r"([0-9.]+)\s*GHz", info["cpu_model"])
        if m:
            info["nominal_ghz"] = float(m.group(1))
            info["nominal_ghz_source"] = "model name"
    if info["nominal_ghz"] is None and info.get("max_ghz"):
        info["nominal_ghz"] = info["max_ghz"]
        info["nominal_ghz_source"] = "lscpu CPU max MHz (no base clock exposed)"
    if info["nominal_ghz"] is None:
        # a virtual machine may expose no frequency but the clock the kernel
        # measured at boot
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("cpu MHz"):
                        info["nominal_ghz"] = round(float(line.split(":")[1]) / 1e3, 3)
                        info["nominal_ghz_source"] = "/proc/cpuinfo cpu MHz (no base clock exposed)"
                        break
        except Exception:
            pass
    return info


def measure(torch, b, args, workload):
    """One workload: W untimed warmup steps, K timed steps (bulk refills + the
    chain launch), the roofline of the chain kernel, and the CPU oracle legs.
    Returns the fields of the bench line for it."""
    import copy
    args = copy.copy(args)
    args.workload = workload
    tuned = None
    if workload in ("gamma", "lda") and not args.no_autotune and not args.window:
        tuned = autotune_launch(torch, b, args)
        args.window, args.wpb = tuned["window"], tuned["wpb"]
    Wk = WORKLOADS[workload](torch, b, args)
    ctx = Wk["ctx"]
    b.brng_set_launch(ctx, args.wpb)
    ev = Events(torch)

    # the bulk refill covers the kinds whose windows the chain kernel reads
    fill_kinds = Wk.get("fill_kinds", Wk["kinds"])

    def step(kpair=None):
        for k in fill_kinds:
            b.brng_fill_base(ctx, k)
        # the chain kernel's own start and end (events the launch records),
        # and the span of the call on the stream (which adds the dispatch gap)
        if kpair is not None:
            b.brng_time_next_launch(ctx, *kpair)
            ev.pairs.setdefault("chains", []).append(kpair)
        e = ev.span("chains_span")
        if "run" in Wk:
            Wk["run"]()
        else:
            b.brng_run_gibbs(ctx, Wk["resume"])
        e.record()

    if "run" in Wk:
        Wk["run"]()
    else:
        b.brng_run_gibbs(ctx, Wk["fresh"])  # fresh start: streams at 0
    for _ in range(max(0, args.warmup - 1)):
        step()
    # kernel event pairs, created (recorded once) before the timed region
    kpairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    for kp in kpairs:
        for e in kp:
            e.record()
    torch.cuda.synchronize()
    ev.pairs.clear()
    cur0 = b.brng_get_cursors(ctx)
    torch.cuda.synchronize()
    # no garbage collection inside the timed region: the steps are queued
    # by this thread, and a long collection would leave the GPU waiting
    import gc
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(args.steps):
        step(kpairs[i])
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gc.enable()
    cur1 = b.brng_get_cursors(ctx)
    ms_step = start.elapsed_time(stop) / args.steps
    value = Wk["deviates"] / (ms_step / 1e3)

    # algorithmic bytes from the entries actually consumed (cursor deltas):
    # each consumed entry is written once and read once; the bulk fill writes
    # the first window of each unit and kind, the chain kernel the rest
    delta = (cur1 - cur0).astype(np.float64) / args.steps  # per step, [unit][kind]
    fill_b = 0.0
    pool_b = 0.0
    for k in Wk["kinds"]:
        eb = Wk["entry_bytes"][k]
        pool_b += 2.0 * eb * delta[:, k].sum()
        if k in fill_kinds:
            fill_b += eb * np.minimum(delta[:, k], Wk["windows"][k]).sum()
    step_b = pool_b + Wk["out_bytes"]
    chain_b = Wk["kernel_bytes"](delta) if "kernel_bytes" in Wk else step_b - fill_b
    chain_ms = float(np.mean(ev.ms("chains")))
    span_ms = float(np.mean(ev.ms("chains_span")))
    gbs = chain_b / (chain_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(Wk["kernel"]),
            "kernel": Wk["kernel"],
            "kernel_ms": round(chain_ms, 4), "call_span_ms": round(span_ms, 4),
            "alg_bytes_per_launch": chain_b}
    out = {
        "value": value,
        "ms_per_step": ms_step,
        "dtype": Wk["dtype"],
        "config": Wk["config"],
        "roofline": roof,
        "step_alg_bytes": step_b,
        "step_hbm_frac": round(step_b / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "entries_per_step": {int(k): float(delta[:, k].sum()) for k in Wk["kinds"]},
        "wall_s": wall,
    }
    if tuned is not None:
        out["autotune"] = {"window": tuned["window"], "wpb": tuned["wpb"],
                           "candidates_ms": {"%d/%d" % (t["window"], t["wpb"]): round(t["seconds"] * 1e3, 4)
                                             for t in tuned["table"]}}
    if "oaat" in Wk and not args.no_oaat:
        out["one_launch_per_step"] = Wk["oaat"](ev)
    b.brng_destroy(ctx)
    if not args.no_cpu:
        # the oracle legs run after every GPU measurement of the run (see
        # run_cpu_legs), so that a pool of host processes never overlaps a
        # timed region
        out["_cpu"] = lambda: cpu_leg(Wk, args)
    return out


def cpu_leg(Wk, args):
    """The oracle on a bounded sample over the host's processes, and on a
    smaller sample in one thread, with the host's description."""
    workers = args.cpu_workers or min(16, os.cpu_count() or 1)
    cb = Wk["cpu"](workers)
    # one core: the same oracle in this process on a smaller sample, and its
    # cycles per deviate at the host's nominal clock (the unit of the paper's
    # results table)
    one = Wk["cpu1"]()
    ghz = args.host["nominal_ghz"]
    if ghz:
        one["cycles_per_deviate_at_nominal"] = round(ghz * 1e9 / one["value"], 1)
    cb["one_core"] = one
    cb.update({k: v for k, v in args.host.items()})
    return cb


def run_cpu_legs(results):
    for r in results:
        leg = r.pop("_cpu", None)
        if leg is not None:
            r["cpu_baseline"] = leg()


HEADLINE = "lda"
EXTRA = ("gamma", "normexp")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="",
                    choices=[""] + sorted(WORKLOADS) + ["served"],
                    help="one workload alone; by default the LDA/Dirichlet workload is the "
                         "headline and the gamma and normal/exponential chains follow under "
                         "'workloads'")
    ap.add_argument("--chains", type=int, default=0)
    ap.add_argument("--chain-steps", type=int, default=0)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--seed", type=int, default=20141217)
    ap.add_argument("--wpb", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--cpu-units", type=int, default=0)
    ap.add_argument("--oaat-steps", type=int, default=100)
    ap.add_argument("--lda-vocab", type=int, default=4096,
                    help="lda_full: vocabulary size")
    ap.add_argument("--lda-topics", type=int, default=64,
                    help="lda_full: topics (1 .. 1,024)")
    ap.add_argument("--no-oaat", action="store_true",
                    help="skip the one-launch-per-step comparison (gamma)")
    ap.add_argument("--served-requests", type=int, default=1000)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="default run: skip the gamma and normal/exponential workloads")
    ap.add_argument("--no-dist", action="store_true",
                    help="skip the per-distribution rates (fill and one-at-a-time calls)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="gamma/lda: use --window/--wpb as given instead of timing candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one conversion of 2^26 words (256 MiB read, 256 MiB "
                         "written): the known-size kernel that scales rocprof's "
                         "FETCH_SIZE/WRITE_SIZE to bytes")
    ap.add_argument("--served-chains-max", type=int, default=65536)
    ap.add_argument("--served-steps-max", type=int, default=10000)
    ap.add_argument("--served-budget-mb", type=int, default=16384)
    ap.add_argument("--served-slots", type=int, default=64)
    ap.add_argument("--served-tick-steps", type=int, default=256)
    ap.add_argument("--served-tick-sweeps", type=int, default=4)
    ap.add_argument("--served-bypass-ms", type=int, default=50,
                    help="served form: later requests that fit may pass a waiting one for "
                         "this long after its arrival")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(each GPU would run its own independent units); use --gpus 1",
              file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_1412_4825_amd import binding as b

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "served":
        served_main(torch, args)
        return
    args.host = host_cpu_info()
    head = args.workload or HEADLINE
    res = measure(torch, b, args, head)
    print("[bench] %s: %.4g deviates/s, roofline %.3f" % (head, res["value"], res["roofline"]["frac"]),
          file=sys.stderr, flush=True)
    out = {
        "metric": "varying-param deviates/s + % HBM roofline",
        "value": res.pop("value"),
        "unit": "deviates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": res.pop("dtype"),
        "data": "synthetic",
        "config": res.pop("config"),
        "roofline": res.pop("roofline"),
    }
    out.update(res)
    # context: what a plain copy reaches on this GPU
    cgbs = copy_bandwidth(torch, b)
    out["roofline"]["copy_gbs"] = round(cgbs, 1)
    out["roofline"]["frac_of_copy"] = round(out["roofline"]["achieved"] / cgbs, 4)
    if not args.workload and not args.no_extra:
        out["workloads"] = {}
        for name in EXTRA:
            r = measure(torch, b, args, name)
            print("[bench] %s: %.4g deviates/s, roofline %.3f" % (name, r["value"], r["roofline"]["frac"]),
                  file=sys.stderr, flush=True)
            out["workloads"][name] = r
    if args.copy_calibration:
        nw = 1 << 26
        words = torch.randint(-2**31, 2**31 - 1, (nw,), dtype=torch.int32, device="cuda")
        conv = torch.empty(nw, dtype=torch.float32, device="cuda")
        b.brng_convert(b.BRNG_U, words, nw, conv, torch.cuda.current_stream())
        torch.cuda.synchronize()
        del words, conv
    if not args.no_dist:
        out["per_distribution"] = per_distribution(torch, b, args)
    if not args.no_served:
        # the metric's second half: served latency and throughput against
        # per-request plain launches on a mixed request stream
        out["served"] = served_section(torch, args, args.served_requests)
    # the CPU oracle legs, once no more GPU work is timed
    run_cpu_legs([out] + list(out.get("workloads", {}).values()))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
