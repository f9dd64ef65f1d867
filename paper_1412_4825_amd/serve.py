"""Request loop for the served form (C interface: brng_serve_*).

`Request` turns one generated request (workloads.served_requests) into the
device arrays and brng_gibbs_desc the library runs; `run_served` drives a
server with requests arriving at given times (continuous batching: arrivals
join at the next tick while earlier requests run); `run_plain` runs the same
requests one launch each, back to back, as the per-request baseline.  Both
leave every request's results in its own device arrays.
"""
from __future__ import annotations

import numpy as np

from . import binding as b

MODEL_OF = {"uniform": b.BRNG_MODEL_TRIANGLE_F64, "normal": b.BRNG_MODEL_NORMEXP,
            "exponential": b.BRNG_MODEL_EXP_CHAIN, "gamma": b.BRNG_MODEL_GAMMA_CHAIN,
            "dirichlet": b.BRNG_MODEL_LDA}


class Request:
    """Device arrays and descriptor of one served request.  The state is
    reset to its initial value by reset()."""

    def __init__(self, torch, q: dict, dev, sums: bool = False):
        self.q = q
        self.model = MODEL_OF[q["kind"]]
        n, s = q["chains"], q["steps"]
        self.keep = []
        if q["kind"] == "uniform":
            self.state = torch.zeros(2 * n, dtype=torch.float64, device=dev)
            self.init = None
            self.deviates = 2 * n * s
        elif q["kind"] in ("normal", "exponential"):
            self.state = torch.zeros(n, dtype=torch.float32, device=dev)
            self.init = None
            self.deviates = (2 if q["kind"] == "normal" else 1) * n * s + n
        elif q["kind"] == "gamma":
            self.init = torch.from_numpy(q["alpha0"]).to(dev)
            self.state = self.init.clone()
            self.deviates = n * s
        else:
            off, ntok = q["offsets"], q["ntok"]
            self.offsets = torch.from_numpy(off).to(dev)
            self.ntok = torch.from_numpy(ntok).to(dev)
            self.init = torch.zeros(int(off[-1]), dtype=torch.int32, device=dev)
            self.state = self.init.clone()
            self.deviates = (int(off[-1]) + int(ntok.sum())) * s
        kw = {}
        if self.model == b.BRNG_MODEL_LDA:
            kw = dict(offsets=self.offsets, ntok=self.ntok)
        # per-chain sums of every output (LDA: per component), the request's
        # summary besides its final state
        self.sums = None
        if sums:
            nout = 4 if q["kind"] in ("uniform", "normal") else 2
            width = int(q["offsets"][-1]) if q["kind"] == "dirichlet" else n
            self.sums = torch.zeros((nout, width), dtype=torch.float64, device=dev)
            kw["sums"] = self.sums
        self.desc = b.gibbs_desc(self.model, n, self.state, max_steps=s, seed=q["seed"], **kw)
        self.units = n if self.model == b.BRNG_MODEL_LDA else (n + 63) // 64

    def reset(self):
        if self.init is None:
            self.state.zero_()
        else:
            self.state.copy_(self.init)
        if self.sums is not None:
            self.sums.zero_()


def run_plain(torch, reqs, window, stream=None):
    """Each request alone, one brng_run_gibbs launch after another on one
    context; returns the per-request device times in seconds (events around
    each launch, the stream drained in between)."""
    n_units = max(r.units for r in reqs)
    ctx = b.brng_create(1, n_units, window, layout=b.BRNG_LAYOUT_ITEMS,
                        stream=stream or torch.cuda.current_stream())
    try:
        out = []
        for r in reqs:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.brng_run_gibbs(ctx, r.desc)
            e1.record()
            e1.synchronize()
            out.append(e0.elapsed_time(e1) / 1e3)
        return np.array(out)
    finally:
        b.brng_destroy(ctx)


def run_served(torch, reqs, arrivals_s, *, budget, window, max_active=64, tick_steps=256,
               tick_sweeps=4, max_bypass_ms=0, stream=None, on_done=None):
    """Serve `reqs`, request i arriving arrivals_s[i] seconds after the start
    (all at 0 for a saturated run).  Returns (latency_s per request, makespan
    seconds from the first arrival to the last completion, server stats).
    on_done(count), if given, is called after each completed request."""
    srv = b.brng_serve_open(budget, window, max_active=max_active, tick_steps=tick_steps,
                            tick_sweeps=tick_sweeps, max_bypass_ms=max_bypass_ms,
                            stream=stream or torch.cuda.current_stream())
    n = len(reqs)
    lat = np.zeros(n)
    try:
        t0 = b.brng_serve_now()
        arr = t0 + (np.asarray(arrivals_s) * 1e9).astype(np.int64)
        index = {}
        i = done = 0
        t_last = t0
        while done < n:
            now = b.brng_serve_now()
            while i < n and arr[i] <= now:
                index[b.brng_serve_submit(srv, reqs[i].desc, int(arr[i]))] = i
                i += 1
            b.brng_serve_progress(srv, wait=(i == n))
            for d in b.brng_serve_poll(srv):
                if d["status"] != 0:
                    raise b.BrngError(d["status"], "served request")
                k = index.pop(d["ticket"])
                lat[k] = (d["t_done_ns"] - d["t_arrive_ns"]) / 1e9
                t_last = max(t_last, d["t_done_ns"])
                done += 1
                if on_done is not None:
                    on_done(done)
        stats = b.brng_serve_stats_get(srv)
    finally:
        b.brng_serve_close(srv)
    return lat, (t_last - arr[0]) / 1e9, stats


def fifo_latency(arrivals_s, service_s):
    """Latency of each request in a single FIFO queue whose server takes
    service_s[i] for request i (the plain per-request form)."""
    t = 0.0
    lat = np.zeros(len(service_s))
    for i, (a, s) in enumerate(zip(arrivals_s, service_s)):
        t = max(t, a) + s
        lat[i] = t - a
    return lat
