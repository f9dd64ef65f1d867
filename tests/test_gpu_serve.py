"""Served form on the GPU: each request's results are the same alone (a plain
brng_run_gibbs) and in a served mix; admission never exceeds the budget; the
time stamps are ordered.  Also the batched form with more requests of one
model than one launch takes.

Every test prints its case before the GPU calls."""
import numpy as np
import pytest

from paper_1412_4825_amd import workloads

pytestmark = pytest.mark.gpu

W_SERVE = [512, 512, 512, 512]      # small windows: many in-kernel refills
W_PLAIN = [4096, 4096, 4096, 4096]  # results do not depend on the window


def _b():
    from paper_1412_4825_amd import binding
    return binding


def _say(*a):
    print("[case]", *a, flush=True)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


N_SUMS = {0: 4, 1: 4, 2: 2, 3: 2, 4: 2}  # outputs x (sum, square) per model


def _requests(dev, sums=False):
    """A mix of every model with traces, uneven lengths and several sizes.
    Returns (descs, arrays-to-check) per request; the arrays are the state and
    traces the request writes (and its sums array when sums=True)."""
    import torch
    b = _b()
    reqs = []

    def add(desc, arrays, keep, width=None):
        if sums:
            w = width if width is not None else desc.n_chains
            sm = torch.zeros((N_SUMS[desc.model], w), dtype=torch.float64, device=dev)
            desc.d_sums = sm.data_ptr()
            arrays = arrays + [sm]
        reqs.append((desc, arrays, keep))

    # triangle, fp64, with both traces
    n, s = 100, 300
    st = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    tx = torch.zeros((s, n), dtype=torch.float64, device=dev)
    ty = torch.zeros((s, n), dtype=torch.float64, device=dev)
    add(b.gibbs_desc(b.BRNG_MODEL_TRIANGLE_F64, n, st, max_steps=s, seed=11, trace=tx, trace2=ty,
                     trace_stride=n), [st, tx, ty], None)
    # normal/exponential chain with both traces
    n, s = 200, 150
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.zeros((s, n), dtype=torch.float32, device=dev)
    te = torch.zeros((s, n), dtype=torch.float32, device=dev)
    add(b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=s, seed=12, trace=ts, trace2=te,
                     trace_stride=n), [st, ts, te], None)
    # gamma chains of uneven lengths, slot order sorted by length
    w = workloads.gamma_chain(n_chains=130, lmin=5, lmax=90, seed=3)
    perm = b.brng_sort_by_length(w["steps"])
    s = int(w["steps"].max())
    st = _t(w["alpha0"], dev)
    tg = torch.full((s, 130), float("nan"), dtype=torch.float32, device=dev)
    keep = (_t(w["steps"], dev), _t(perm, dev), st.clone())
    add(b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 130, st, max_steps=s, seed=13, trace=tg,
                     trace_stride=130, steps=keep[0], perm=keep[1]), [st, tg], keep)
    # exponential chain
    n, s = 70, 257
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    tr = torch.zeros((s, n), dtype=torch.float32, device=dev)
    add(b.gibbs_desc(b.BRNG_MODEL_EXP_CHAIN, n, st, max_steps=s, seed=14, trace=tr,
                     trace_stride=n), [st, tr], None)
    # LDA documents of every K
    wl = workloads.lda(n_docs=20, sweeps=7, seed=6)
    tot = int(wl["offsets"][-1])
    cnt = torch.zeros(tot, dtype=torch.int32, device=dev)
    th = torch.zeros((7, tot), dtype=torch.float32, device=dev)
    ct = torch.zeros((7, tot), dtype=torch.int32, device=dev)
    keep = (_t(wl["offsets"], dev), _t(wl["ntok"], dev))
    add(b.gibbs_desc(b.BRNG_MODEL_LDA, 20, cnt, max_steps=7, seed=15, trace=th, trace2=ct,
                     trace_stride=tot, offsets=keep[0], ntok=keep[1]), [cnt, th, ct], keep,
        width=tot)
    # a second, larger gamma request (several units)
    w2 = workloads.gamma_chain(n_chains=700, lmin=30, lmax=60, seed=8)
    st2 = _t(w2["alpha0"], dev)
    keep2 = (_t(w2["steps"], dev), st2.clone())
    add(b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 700, st2, max_steps=60, seed=16,
                     steps=keep2[0]), [st2], keep2)
    return reqs


def _alone(dev, desc, arrays, keep):
    """Run one request by itself with the plain call; return copies of its
    arrays."""
    import torch
    b = _b()
    layout = 1 if desc.model == b.BRNG_MODEL_LDA else 0
    ctx = b.brng_create(desc.seed, desc.n_chains, W_PLAIN, layout=layout,
                        stream=torch.cuda.current_stream())
    try:
        b.brng_run_gibbs(ctx, desc)
        return [_np(a).copy() for a in arrays]
    finally:
        b.brng_destroy(ctx)


@pytest.mark.parametrize("sums", [False, True], ids=["plain", "sums"])
def test_served_equals_alone(dev, sums):
    import torch
    b = _b()
    _say("serve alone-vs-mix: 6 requests, 5 models, sums", sums)
    alone = []
    for desc, arrays, keep in _requests(dev, sums):
        alone.append(_alone(dev, desc, arrays, keep))
    mix = _requests(dev, sums)
    budget = 3 * 1024 * 1024  # room for a few requests at a time
    srv = b.brng_serve_open(budget, W_SERVE, max_active=3, tick_steps=16, tick_sweeps=2,
                            stream=torch.cuda.current_stream())
    try:
        tickets = [b.brng_serve_submit(srv, d) for d, _, _ in mix]
        done = []
        while len(done) < len(mix):
            b.brng_serve_progress(srv, wait=True)
            st = b.brng_serve_stats_get(srv)
            assert st["bytes_in_use"] <= budget and st["active"] <= 3
            done += b.brng_serve_poll(srv)
        st = b.brng_serve_stats_get(srv)
        print("serve stats", st, flush=True)
        assert st["bytes_peak"] <= budget and st["ticks"] > 10
        assert sorted(d["ticket"] for d in done) == sorted(tickets)
        for d in done:
            assert d["status"] == 0
            assert d["t_arrive_ns"] <= d["t_admit_ns"] <= d["t_done_ns"]
    finally:
        b.brng_serve_close(srv)
    for i, ((desc, arrays, _), ref) in enumerate(zip(mix, alone)):
        for j, (a, r) in enumerate(zip(arrays, ref)):
            got = _np(a)
            assert np.array_equal(got.view(np.uint8), r.view(np.uint8)), (i, desc.model, j)


def test_serve_rejects_and_admits_by_footprint(dev):
    import torch
    b = _b()
    _say("serve admission")
    srv = b.brng_serve_open(1 << 20, W_SERVE, max_active=8, tick_steps=8, tick_sweeps=1,
                            stream=torch.cuda.current_stream())
    try:
        # 200 units x 2 kinds x 512 floats = 800 KiB of pools: fits alone
        n = 200 * 64
        sts = [torch.ones(n, dtype=torch.float32, device=dev) for _ in range(3)]
        ds = [b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, sts[i], max_steps=20, seed=100 + i)
              for i in range(3)]
        big = torch.ones(400 * 64, dtype=torch.float32, device=dev)
        with pytest.raises(b.BrngError) as e:
            b.brng_serve_submit(srv, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 400 * 64, big,
                                                  max_steps=5, seed=1))
        assert e.value.status == b.BRNG_E_NOMEM
        with pytest.raises(b.BrngError) as e:
            b.brng_serve_submit(srv, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 64, big,
                                                  max_steps=5, seed=1, flags=1))
        assert e.value.status == b.BRNG_E_ARG
        for d in ds:
            b.brng_serve_submit(srv, d)
        seen_active = []
        done = []
        while len(done) < 3:
            b.brng_serve_progress(srv, wait=True)
            st = b.brng_serve_stats_get(srv)
            seen_active.append(st["active"])
            assert st["bytes_in_use"] <= (1 << 20)
            done += b.brng_serve_poll(srv)
        # one request's footprint is more than half the budget: one at a time
        assert max(seen_active) <= 1
        assert [d["ticket"] for d in done] == [1, 2, 3]
    finally:
        b.brng_serve_close(srv)


def test_batched_many_requests_equal_alone(dev):
    """More requests of one model than one launch holds (16): every request
    equals its plain run."""
    import torch
    b = _b()
    _say("batched: 21 gamma requests in one call")
    n_req, per = 21, 90
    ws = [workloads.gamma_chain(n_chains=per + 7 * i, lmin=3, lmax=40, seed=50 + i)
          for i in range(n_req)]
    refs = []
    for i, w in enumerate(ws):
        st = _t(w["alpha0"], dev)
        tg = torch.full((40, w["n_chains"]), float("nan"), dtype=torch.float32, device=dev)
        d = b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, w["n_chains"], st, max_steps=40,
                         seed=500 + i, trace=tg, trace_stride=w["n_chains"],
                         steps=_t(w["steps"], dev))
        refs.append(_alone(dev, d, [st, tg], None))
    units = [(w["n_chains"] + 63) // 64 for w in ws]
    ctx = b.brng_create(9, 64 * (sum(units) + n_req), [0, 512, 512, 0],
                        stream=torch.cuda.current_stream())
    try:
        descs, outs, base = [], [], 0
        keep = []
        for i, w in enumerate(ws):
            st = _t(w["alpha0"], dev)
            tg = torch.full((40, w["n_chains"]), float("nan"), dtype=torch.float32, device=dev)
            stp = _t(w["steps"], dev)
            keep.append(stp)
            descs.append(b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, w["n_chains"], st, max_steps=40,
                                      seed=500 + i, trace=tg, trace_stride=w["n_chains"],
                                      steps=stp, unit_base=base))
            outs.append((st, tg))
            base += units[i] + 1
        b.brng_run_gibbs(ctx, descs)
        for i, ((st, tg), ref) in enumerate(zip(outs, refs)):
            assert np.array_equal(_np(st), ref[0]), i
            assert np.array_equal(_np(tg), ref[1], equal_nan=True), i
    finally:
        b.brng_destroy(ctx)


def test_launch_shape_invariance_and_graph_replay(dev):
    """Waves per workgroup change nothing; the batched form captured in a
    graph (bulk refills + one multi-request launch) replays to the same bits
    as the same calls made eagerly, with eager work between replays."""
    import torch
    b = _b()
    _say("launch shape 1/2/4/8 and graph replay")
    w = workloads.gamma_chain(n_chains=300, lmin=10, lmax=40, seed=21)
    outs = []
    for wpb in (1, 2, 4, 8):
        ctx = b.brng_create(5, 300, [0, 512, 512, 0], stream=torch.cuda.current_stream())
        try:
            b.brng_set_launch(ctx, wpb)
            st = _t(w["alpha0"], dev)
            tg = torch.full((40, 300), float("nan"), dtype=torch.float32, device=dev)
            b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 300, st, max_steps=40,
                                               seed=5, trace=tg, trace_stride=300,
                                               steps=_t(w["steps"], dev)))
            outs.append((_np(st), _np(tg)))
        finally:
            b.brng_destroy(ctx)
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1], equal_nan=True)

    # graph: two requests (gamma + normal/exponential) resumed per replay
    n1, n2, steps = 300, 200, 16

    def make(stream):
        ctx = b.brng_create(6, n1 + n2 + 64, [0, 1024, 1024, 0], stream=stream)
        st1 = _t(w["alpha0"], dev)
        st2 = torch.zeros(n2, dtype=torch.float32, device=dev)
        t1 = torch.zeros((steps, n1), dtype=torch.float32, device=dev)
        t2 = torch.zeros((steps, n2), dtype=torch.float32, device=dev)
        base2 = (n1 + 63) // 64

        def descs(flags):
            return [b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n1, st1, max_steps=steps, seed=61,
                                 trace=t1, trace_stride=n1, flags=flags),
                    b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n2, st2, max_steps=steps, seed=62,
                                 trace=t2, trace_stride=n2, unit_base=base2, flags=flags)]
        return ctx, (st1, st2, t1, t2), descs

    ref = []
    ctx, arrs, descs = make(torch.cuda.current_stream())
    try:
        b.brng_run_gibbs(ctx, descs(0))
        for _ in range(3):
            b.brng_fill_base(ctx, b.BRNG_N)
            b.brng_fill_base(ctx, b.BRNG_E)
            b.brng_run_gibbs(ctx, descs(b.BRNG_FLAG_RESUME))
            ref.append([_np(a).copy() for a in arrs])
    finally:
        b.brng_destroy(ctx)
    s = torch.cuda.Stream()
    ctx, arrs, descs = make(s)
    try:
        with torch.cuda.stream(s):
            b.brng_run_gibbs(ctx, descs(0))
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        rd = descs(b.BRNG_FLAG_RESUME)
        with torch.cuda.graph(g, stream=s):
            b.brng_fill_base(ctx, b.BRNG_N)
            b.brng_fill_base(ctx, b.BRNG_E)
            b.brng_run_gibbs(ctx, rd)
        junk = torch.zeros(1 << 20, device=dev)
        for i in range(3):
            g.replay()
            torch.cuda.synchronize()
            got = [_np(a) for a in arrs]
            for a, r in zip(got, ref[i]):
                assert np.array_equal(a, r), i
            junk.add_(1.0)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        b.brng_destroy(ctx)


def _sums_from_trace(model, n, tr, tr2, steps=None, perm=None):
    """Per-chain sums of the outputs recomputed from the traces in step
    order (fp64, one rounding per add; v * v is exact for fp32 v and rounded
    once for fp64 v, as the kernels compute it).  Gamma traces are
    [step][slot] with slot -> chain by perm and steps per chain."""
    outs = [tr] if tr2 is None else [tr, tr2]
    res = []
    for o in outs:
        o = o.astype(np.float64)
        T = o.shape[0]
        s1 = np.zeros(o.shape[1])
        s2 = np.zeros(o.shape[1])
        for t in range(T):
            v = o[t]
            if steps is not None:
                ok = t < steps
                v = np.where(ok, v, 0.0)
            s1 = s1 + v
            s2 = s2 + v * v
        res += [s1, s2]
    out = np.stack(res)
    if perm is not None:  # slot order -> chain order
        u = np.empty_like(out)
        u[:, perm] = out
        out = u
    return out


def test_sums_equal_trace_recomputation(dev):
    """Every model's sums equal the same sums recomputed from its trace bit
    for bit, and a run split in two launches gives the sums of one."""
    import torch
    b = _b()
    _say("sums against traces, every model")
    for desc, arrays, keep in _requests(dev, sums=True):
        model = desc.model
        layout = 1 if model == b.BRNG_MODEL_LDA else 0
        ctx = b.brng_create(desc.seed, desc.n_chains, W_SERVE, layout=layout,
                            stream=torch.cuda.current_stream())
        try:
            b.brng_run_gibbs(ctx, desc)
            got = [_np(a) for a in arrays]
        finally:
            b.brng_destroy(ctx)
        sm = got[-1]
        if model == b.BRNG_MODEL_TRIANGLE_F64:
            ref = _sums_from_trace(model, desc.n_chains, got[1], got[2])
        elif model == b.BRNG_MODEL_NORMEXP:
            ref = _sums_from_trace(model, desc.n_chains, got[1], got[2])
        elif model == b.BRNG_MODEL_EXP_CHAIN:
            ref = _sums_from_trace(model, desc.n_chains, got[1], None)
        elif model == b.BRNG_MODEL_LDA:
            th = got[1]
            ref = _sums_from_trace(model, th.shape[1], th, None)
        else:
            if len(got) < 3:  # the gamma request without a trace
                continue
            stp = keep[0].cpu().numpy()
            perm = keep[1].cpu().numpy()
            ref = _sums_from_trace(model, desc.n_chains, got[1], None, steps=stp[perm], perm=perm)
        assert np.array_equal(sm.view(np.uint64), ref.view(np.uint64)), model
    # split: normal/exponential 40 + 60 steps (resumed) = 100 steps at once
    n = 130
    outs = []
    for split in (False, True):
        ctx = b.brng_create(5, n, [0, 512, 512, 0], stream=torch.cuda.current_stream())
        try:
            st = torch.zeros(n, dtype=torch.float32, device=dev)
            sm = torch.zeros((4, n), dtype=torch.float64, device=dev)
            if split:
                b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=40,
                                                   seed=5, sums=sm))
                b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=60,
                                                   seed=5, sums=sm, flags=b.BRNG_FLAG_RESUME))
            else:
                b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, max_steps=100,
                                                   seed=5, sums=sm))
            outs.append((_np(st), _np(sm)))
        finally:
            b.brng_destroy(ctx)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1].view(np.uint64), outs[1][1].view(np.uint64))


def test_batched_mixed_models_one_call(dev):
    """120 requests of all five models (some with sums) in one
    brng_run_gibbs call: one launch over all their units, each wave running
    its request's model; every request equals its plain run bit for bit."""
    import torch
    b = _b()
    _say("batched: 120 mixed requests in one call")
    rng = np.random.default_rng(77)
    specs = []
    for i in range(120):
        model = i % 5
        specs.append((model, int(rng.integers(1, 200)), int(rng.integers(3, 30)), 900 + i,
                      bool(i % 3 == 0)))

    def build(model, n, s, seed, with_sums, unit_base):
        if model == b.BRNG_MODEL_TRIANGLE_F64:
            st = torch.zeros(2 * n, dtype=torch.float64, device=dev)
            tr = torch.zeros((s, n), dtype=torch.float64, device=dev)
            d = b.gibbs_desc(model, n, st, max_steps=s, seed=seed, trace=tr, trace_stride=n,
                             unit_base=unit_base)
            arrs, keep, units, width = [st, tr], None, (n + 63) // 64, n
        elif model in (b.BRNG_MODEL_NORMEXP, b.BRNG_MODEL_EXP_CHAIN):
            st = torch.zeros(n, dtype=torch.float32, device=dev)
            tr = torch.zeros((s, n), dtype=torch.float32, device=dev)
            d = b.gibbs_desc(model, n, st, max_steps=s, seed=seed, trace=tr, trace_stride=n,
                             unit_base=unit_base)
            arrs, keep, units, width = [st, tr], None, (n + 63) // 64, n
        elif model == b.BRNG_MODEL_GAMMA_CHAIN:
            w = workloads.gamma_chain(n_chains=n, lmin=1, lmax=s, seed=seed)
            st = _t(w["alpha0"], dev)
            stp = _t(w["steps"], dev)
            tr = torch.full((s, n), float("nan"), dtype=torch.float32, device=dev)
            d = b.gibbs_desc(model, n, st, max_steps=s, seed=seed, trace=tr, trace_stride=n,
                             steps=stp, unit_base=unit_base)
            arrs, keep, units, width = [st, tr], stp, (n + 63) // 64, n
        else:
            nd = max(1, n // 20)
            wl = workloads.lda(n_docs=nd, sweeps=s, seed=seed)
            tot = int(wl["offsets"][-1])
            cnt = torch.zeros(tot, dtype=torch.int32, device=dev)
            th = torch.zeros((s, tot), dtype=torch.float32, device=dev)
            keep = (_t(wl["offsets"], dev), _t(wl["ntok"], dev))
            d = b.gibbs_desc(model, nd, cnt, max_steps=s, seed=seed, trace=th, trace_stride=tot,
                             offsets=keep[0], ntok=keep[1], unit_base=unit_base)
            arrs, units, width = [cnt, th], nd, tot
        if with_sums:
            sm = torch.zeros((N_SUMS[model], width), dtype=torch.float64, device=dev)
            d.d_sums = sm.data_ptr()
            arrs = arrs + [sm]
        return d, arrs, keep, units

    refs = []
    for model, n, s, seed, ws in specs:
        d, arrs, keep, _ = build(model, n, s, seed, ws, 0)
        refs.append(_alone(dev, d, arrs, keep))
    descs, outs, keeps, base = [], [], [], 0
    for model, n, s, seed, ws in specs:
        d, arrs, keep, units = build(model, n, s, seed, ws, base)
        descs.append(d)
        outs.append(arrs)
        keeps.append(keep)
        base += units
    ctx = b.brng_create(3, base, W_PLAIN, layout=1, stream=torch.cuda.current_stream())
    try:
        b.brng_run_gibbs(ctx, descs)
        for i, (arrs, ref) in enumerate(zip(outs, refs)):
            for j, (a, r) in enumerate(zip(arrs, ref)):
                got = _np(a)
                assert np.array_equal(got.view(np.uint8), r.view(np.uint8)), (i, specs[i], j)
    finally:
        b.brng_destroy(ctx)


def test_admission_passes_a_blocked_head(dev):
    """With a bypass bound, a small request that fits is admitted while an
    older large one waits for memory; with none, it waits behind it."""
    import torch
    b = _b()
    _say("serve admission past a blocked head")
    n_big = 150 * 64  # 150 units x (2 x 512 floats + 96 B) ~ 0.6 MiB
    for bypass in (0, 60000):
        srv = b.brng_serve_open(1 << 20, W_SERVE, max_active=8, tick_steps=8, tick_sweeps=1,
                                max_bypass_ms=bypass, stream=torch.cuda.current_stream())
        try:
            sts = [torch.ones(n_big, dtype=torch.float32, device=dev) for _ in range(2)]
            small = torch.ones(64, dtype=torch.float32, device=dev)
            t = [b.brng_serve_submit(srv, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n_big, sts[i],
                                                       max_steps=400, seed=200 + i))
                 for i in range(2)]
            t.append(b.brng_serve_submit(srv, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, 64, small,
                                                           max_steps=5, seed=300)))
            done = {}
            while len(done) < 3:
                b.brng_serve_progress(srv, wait=True)
                for d in b.brng_serve_poll(srv):
                    assert d["status"] == 0
                    done[d["ticket"]] = d
            admit = [done[k]["t_admit_ns"] for k in t]
            if bypass:
                assert admit[2] < admit[1], admit  # the small one went first
            else:
                assert admit[0] <= admit[1] <= admit[2], admit
        finally:
            b.brng_serve_close(srv)
