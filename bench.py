#!/usr/bin/env python3
"""Benchmark of the varying-parameter pool RNG on one MI355X.

Default workload (normal/exponential chains): 65,536 chains x 1,000 steps,
s' ~ N(0.9 s, 0.5 + |s|) then e ~ Exp(1 + s'^2), fp32, Philox4x32-10 pools
with a window of 4,096 entries per unit (64 chains) per kind, refilled on
exhaustion.  One timed step is the whole hot path over that batch: bulk
refill of the Gaussian and exponential windows (one 128-bit store per Philox
block) followed by one launch that runs every chain for all 1,000 steps from
the pools (regenerating each window in place when it runs out), writing both
outputs of every step.  Chains continue from step to step.

Prints one JSON line: deviates/s, the roofline of the dominant kernel
(algorithmic bytes over its event-timed duration against 8 TB/s), and the
CPU oracle timed on the host over the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _round_up(x, m):
    return (x + m - 1) // m * m


class Timer:
    """HIP events on the library's stream, per named kernel launch."""

    def __init__(self, torch):
        self.torch = torch
        self.marks = []

    def mark(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.marks.append((name, e))

    def per_name(self):
        out = {}
        for (name, a), (_, b) in zip(self.marks[:-1], self.marks[1:]):
            if name is None:
                continue
            out.setdefault(name, []).append(a.elapsed_time(b))
        return out


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def setup_normexp(torch, b, args):
    n, steps = args.chains or 65536, args.chain_steps or 1000
    # pool window per unit (64 chains) per kind: 4,096 entries, refilled on
    # exhaustion inside the chain kernel
    W = args.window or 4096
    dev = torch.device("cuda:0")
    ctx = b.brng_create(args.seed, n, [0, W, W, 0], stream=torch.cuda.current_stream())
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.empty((steps, n), dtype=torch.float32, device=dev)
    te = torch.empty((steps, n), dtype=torch.float32, device=dev)
    fresh = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=steps, seed=args.seed,
                         trace=ts, trace2=te, trace_stride=n)
    resume = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=steps, seed=args.seed,
                          trace=ts, trace2=te, trace_stride=n, flags=b.BRNG_FLAG_RESUME)
    units = (n + 63) // 64
    state = {"first": True}

    def step(timer):
        if state["first"]:
            # fresh start: streams at 0, s_0 is each chain's first Gaussian
            timer.mark(None)
            b.brng_run_gibbs(ctx, fresh)
            state["first"] = False
            timer.mark(None)
            return
        timer.mark("fill")
        b.brng_fill_base(ctx, b.BRNG_N)
        b.brng_fill_base(ctx, b.BRNG_E)
        timer.mark("chains")
        b.brng_run_gibbs(ctx, resume)
        timer.mark(None)

    deviates = 2 * n * steps
    consumed = 2 * n * steps  # one N and one E entry per chain-step
    # algorithmic bytes: every consumed pool entry is written once and read
    # once (4 B each), every output is written once (4 B).  The bulk fill
    # writes the first window of each unit and kind; the chain kernel writes
    # the rest (its in-kernel refills) and does all reads and output writes.
    per_unit_kind = 64 * steps
    fill_written = 2 * units * min(W, per_unit_kind)
    bytes_ = {
        "fill": fill_written * 4,
        "chains": (consumed - fill_written) * 4 + consumed * 4 + deviates * 4,
    }
    launches = {"fill": 2, "chains": 1}
    cfg = {"workload": "normal/exponential chains: s'~N(0.9s,0.5+|s|), e~Exp(1+s'^2)",
           "chains": n, "steps": steps, "window_per_unit_per_kind": W, "unit_chains": 64,
           "precision": "fp32", "generator": "Philox4x32-10"}

    def cpu(workers):
        return cpu_normexp(args.seed, n, steps, workers)

    return dict(ctx=ctx, step=step, deviates=deviates, bytes=bytes_, launches=launches,
                config=cfg, cpu=cpu, dtype="f32",
                kernels={"fill": "k_fill", "chains": "k_gibbs<NORMEXP>"})


def _normexp_slice(args):
    seed, unit0, n, steps = args
    import oracle
    t = time.perf_counter()
    oracle.normexp(seed, n, steps, unit0=unit0)
    return time.perf_counter() - t


def cpu_normexp(seed, n, steps, workers):
    """The oracle over the whole workload, unit ranges split across processes."""
    import multiprocessing as mp

    units = (n + 63) // 64
    per = (units + workers - 1) // workers
    jobs = []
    for w in range(workers):
        u0, u1 = w * per, min(units, (w + 1) * per)
        if u0 >= u1:
            continue
        jobs.append((seed, u0, min(n, u1 * 64) - u0 * 64, steps))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        busy = pool.map(_normexp_slice, jobs)
    wall = time.perf_counter() - t0
    dev = 2 * n * steps
    return {"value": dev / wall, "unit": "deviates/s", "cores": len(jobs), "kind": "oracle",
            "sample": "whole workload (%d chains x %d steps, %.2e deviates) split by unit "
                      "over %d processes; %.1f s of CPU work" % (n, steps, dev, len(jobs),
                                                                 sum(busy))}


WORKLOADS = {"normexp": setup_normexp}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="normexp", choices=sorted(WORKLOADS))
    ap.add_argument("--chains", type=int, default=0)
    ap.add_argument("--chain-steps", type=int, default=0)
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--seed", type=int, default=20141217)
    ap.add_argument("--wpb", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0)
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
    W = WORKLOADS[args.workload](torch, b, args)
    b.brng_set_launch(W["ctx"], args.wpb)
    step = W["step"]

    warm = Timer(torch)
    for _ in range(max(1, args.warmup)):
        step(warm)
    torch.cuda.synchronize()
    timer = Timer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step(timer)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps
    value = W["deviates"] / (ms_step / 1e3)

    per = timer.per_name()
    kern = {}
    for name, times in per.items():
        avg_ms = sum(times) / len(times) / W["launches"][name]
        gbs = W["bytes"][name] / W["launches"][name] / (avg_ms / 1e3) / 1e9
        kern[name] = {"kernel": W["kernels"][name], "ms_per_launch": avg_ms,
                      "launches_per_step": W["launches"][name],
                      "alg_bytes_per_launch": W["bytes"][name] / W["launches"][name],
                      "GBps": gbs}
    dom = max(kern, key=lambda k: kern[k]["ms_per_launch"] * kern[k]["launches_per_step"])
    roof = {"bound": "hbm", "achieved": round(kern[dom]["GBps"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(kern[dom]["GBps"] / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": kern[dom]["kernel"]}
    step_bytes = sum(W["bytes"].values())
    out = {
        "metric": "varying-param deviates/s + % HBM roofline",
        "value": value,
        "unit": "deviates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": W["dtype"],
        "data": "synthetic",
        "config": W["config"],
        "roofline": roof,
        "step_alg_bytes": step_bytes,
        "step_hbm_frac": round(step_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kern,
        "wall_s": wall,
    }
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = W["cpu"](workers)
    b.brng_destroy(W["ctx"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
