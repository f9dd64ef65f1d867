"""Parity at the benchmark's full sizes and launch configuration, on sampled
units the oracle computes one by one: the fresh launch and then a resumed
launch after the bulk refills, as bench.py times it.

- normal/exponential chains: 65,536 chains x 1,000 steps, window 4,096;
- gamma chains: 262,144 chains of lengths U{50..1000}, slots sorted by
  length, window 512, eight waves per block requested (the autotuner's usual
  choice; the launch fits four in its LDS);
- LDA: 16,384 documents x 100 sweeps, window 512, eight waves per block
  requested.

Every test prints its case before the GPU calls."""
import numpy as np
import pytest

import oracle
from paper_1412_4825_amd import workloads
from tests.parity_util import compare_rounds, compare_units, within

pytestmark = pytest.mark.gpu

SEED = 20141217


def _b():
    from paper_1412_4825_amd import binding
    return binding


def _say(*a):
    print("[case]", *a, flush=True)


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _cols(t, cols):
    """Columns of a [row][col] device array, to the host."""
    import torch
    idx = torch.as_tensor(np.asarray(cols, dtype=np.int64), device=t.device)
    out = t.index_select(1, idx).cpu().numpy()
    torch.cuda.synchronize()
    return out


def test_normexp_full_size(dev):
    import torch
    b = _b()
    n, steps, W = 65536, 1000, 4096
    _say("normexp full size", n, steps, W)
    ctx = b.brng_create(SEED, n, [0, W, W, 0], stream=torch.cuda.current_stream())
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    te = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    units = [0, 1, 511, 777, 1023]
    try:
        # the starting states the fresh run draws (entries 0..63 of each
        # sampled unit's Gaussian window, filled by brng_create)
        s_first = np.concatenate([b.brng_get_window(ctx, b.BRNG_N, u)[2][:64] for u in units])
        b.brng_set_launch(ctx, 4)
        kw = dict(max_steps=steps, seed=SEED, trace=ts, trace2=te, trace_stride=n)
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, **kw))
        runs = [(_cols(ts, [64 * u + c for u in units for c in range(64)]),
                 _cols(te, [64 * u + c for u in units for c in range(64)]))]
        s_mid = st.cpu().numpy().copy()
        b.brng_fill_base(ctx, b.BRNG_N)
        b.brng_fill_base(ctx, b.BRNG_E)
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n, st, flags=b.BRNG_FLAG_RESUME,
                                           **kw))
        runs.append((_cols(ts, [64 * u + c for u in units for c in range(64)]),
                     _cols(te, [64 * u + c for u in units for c in range(64)])))
        cur = b.brng_get_cursors(ctx)
    finally:
        b.brng_destroy(ctx)
    # the gate: per-step replay from the GPU's own states, both launches,
    # every output at the single-result bar
    for i, u in enumerate(units):
        sl = slice(64 * i, 64 * i + 64)
        starts = (s_first[sl], s_mid[64 * u:64 * u + 64])
        qcur = None
        for k, (gs, ge) in enumerate(runs):
            s_in = np.vstack([starts[k][None, :], gs[:-1, sl]])
            q = oracle.normexp_replay(SEED, s_in, gs[:, sl], k == 0, cursors=qcur, unit0=u)
            qcur = q["cursors"]
            if k == 0:
                assert within(starts[0], q["s0"], q["s0tol"]).all(), u
            for g, ref, tol, name in ((gs[:, sl], q["strace"], q["stol"], "s"),
                                      (ge[:, sl], q["etrace"], q["etol"], "e")):
                ok = within(g, ref, tol)
                if not ok.all():
                    t, c = np.argwhere(~ok)[0]
                    print("normexp replay mismatch unit", u, "run", k, name, "step", t, "chain",
                          c, "gpu", g[t, c], "ref", ref[t, c], "tol", tol[t, c], "count",
                          int((~ok).sum()), flush=True)
                assert ok.all(), (u, k, name)
        assert np.array_equal(cur[u], qcur[0]), u
    # free-running against the fp64 chains (bounds propagated along them)
    for i, u in enumerate(units):
        sl = slice(64 * i, 64 * i + 64)
        r1 = oracle.normexp(SEED, 64, steps, unit0=u)
        # the resumed launch starts from the GPU's own fp32 state (replay)
        r2 = oracle.normexp(SEED, 64, steps, s0=s_mid[64 * u:64 * u + 64], cursors=r1["cursors"],
                            unit0=u)
        for k, ((gs, ge), r) in enumerate(zip(runs, (r1, r2))):
            for g, ref, tol, name in ((gs[:, sl], r["strace"], r["stol"], "s"),
                                      (ge[:, sl], r["etrace"], r["etol"], "e")):
                ok = within(g, ref, tol)
                if not ok.all():
                    t, c = np.argwhere(~ok)[0]
                    print("normexp mismatch unit", u, "run", k, name, "step", t, "chain", c,
                          "gpu", g[t, c], "ref", ref[t, c], "tol", tol[t, c],
                          "count", int((~ok).sum()), flush=True)
                    lo = max(0, t - 2)
                    print(" s", gs[lo:t + 1, sl][:, c], r["strace"][lo:t + 1, c], flush=True)
                assert ok.all(), (u, k, name)
        assert np.array_equal(cur[u], r2["cursors"][0]), u


def test_gamma_full_size(dev):
    import torch
    b = _b()
    w = workloads.gamma_chain(n_chains=262144, seed=SEED)
    n, W = w["n_chains"], 512
    perm = b.brng_sort_by_length(w["steps"])
    smax = int(w["steps"].max())
    _say("gamma full size", n, smax, W)
    ctx = b.brng_create(SEED, n, [0, W, W, 0], stream=torch.cuda.current_stream())
    st = _t(w["alpha0"], dev)
    tg = torch.full((smax, n), float("nan"), dtype=torch.float32, device=dev)
    units = [0, 1, 1024, 2047, 3000, 4095]
    cols = [64 * u + c for u in units for c in range(64)]
    try:
        b.brng_set_launch(ctx, 8)
        kw = dict(max_steps=smax, seed=SEED, trace=tg, trace_stride=n,
                  steps=_t(w["steps"], dev), perm=_t(perm, dev))
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st, **kw))
        runs = [_cols(tg, cols)]
        a_mid = st.cpu().numpy().copy()
        b.brng_fill_base(ctx, b.BRNG_N)
        b.brng_fill_base(ctx, b.BRNG_E)
        tg.fill_(float("nan"))
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st,
                                           flags=b.BRNG_FLAG_RESUME, **kw))
        runs.append(_cols(tg, cols))
        cur = b.brng_get_cursors(ctx)
    finally:
        b.brng_destroy(ctx)
    # the gate: every draw replayed from the shape the GPU formed for it
    replay_flips = 0
    for i, u in enumerate(units):
        chains = perm[64 * u:64 * u + 64]
        ident = np.arange(64, dtype=np.int32)
        sl = slice(64 * i, 64 * i + 64)
        qcur = None
        for k, (g, a0) in enumerate(zip(runs, (w["alpha0"][chains], a_mid[chains]))):
            shape = oracle.chain_shapes_fp32(a0, g[:, sl])
            q = oracle.gamma_chain_replay(SEED, shape, w["steps"][chains], perm=ident,
                                          cursors=qcur, unit0=u)
            qcur = q["cursors"]
            bad, flips = compare_rounds(g[:, sl], q["gtrace"], q["gtol"], q["gmargin"], q["gr0"],
                                        q["gr1"], np.zeros(64, dtype=np.int64))
            if bad:
                ok = within(g[:, sl], q["gtrace"], q["gtol"]) | (q["gr1"] < 0)
                rb = q["gr1"][~ok].min()
                tt, c = np.argwhere(~ok & (q["gr1"] == rb))[0]
                print("gamma replay mismatch unit", u, "run", k, "round", rb, "step", tt, "slot",
                      c, "gpu", g[tt, sl][c], "ref", q["gtrace"][tt, c], "tol", q["gtol"][tt, c],
                      "margin", q["gmargin"][tt, c], flush=True)
            assert bad == 0, (u, k)
            replay_flips += len(flips)
            if flips:
                break
        else:
            assert np.array_equal(cur[u], qcur[0]), u
    print("gamma full-size replay flips", replay_flips, flush=True)
    assert replay_flips <= 2
    # free-running against the fp64 chains (shape bounds propagated)
    flips_total = 0
    for i, u in enumerate(units):
        chains = perm[64 * u:64 * u + 64]
        ident = np.arange(64, dtype=np.int32)
        r1 = oracle.gamma_chain(SEED, w["alpha0"][chains], w["steps"][chains], perm=ident, unit0=u)
        # the resumed launch starts from the GPU's own fp32 shapes (replay)
        r2 = oracle.gamma_chain(SEED, a_mid[chains], w["steps"][chains], perm=ident,
                                cursors=r1["cursors"], unit0=u)
        sl = slice(64 * i, 64 * i + 64)
        for g, r in zip(runs, (r1, r2)):
            t = r["gtrace"].shape[0]
            bad, flips = compare_rounds(g[:t, sl], r["gtrace"], r["gtol"], r["gmargin"],
                                        r["gr0"], r["gr1"], np.zeros(64, dtype=np.int64))
            if bad:
                ok = within(g[:t, sl], r["gtrace"], r["gtol"]) | (r["gr1"] < 0)
                rb = r["gr1"][~ok].min()
                tt, c = np.argwhere(~ok & (r["gr1"] == rb))[0]
                print("gamma mismatch unit", u, "round", rb, "step", tt, "slot", c, "gpu",
                      g[tt, sl][c], "ref", r["gtrace"][tt, c], "tol", r["gtol"][tt, c], "margin",
                      r["gmargin"][tt, c], flush=True)
            assert bad == 0, u
            flips_total += len(flips)
            if flips:
                break  # the unit's course changed at a permitted flip
        else:
            assert np.array_equal(cur[u], r2["cursors"][0]), u
    print("gamma full-size flips", flips_total, flush=True)
    assert flips_total <= 2


def test_expchain_full_size(dev):
    """Exponential chains (the served exponential kind) at the served
    stream's largest request: 65,536 chains x 10,000 steps, window 4,096,
    a fresh launch then a resumed one, replayed on sampled units."""
    import torch
    b = _b()
    n, steps, W = 65536, 10000, 4096
    _say("expchain full size", n, steps, W)
    ctx = b.brng_create(SEED, n, [0, 0, W, 0], stream=torch.cuda.current_stream())
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    te = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    units = [0, 3, 600, 1023]
    cols = [64 * u + c for u in units for c in range(64)]
    try:
        e_first = np.concatenate([b.brng_get_window(ctx, b.BRNG_E, u)[2][:64] for u in units])
        b.brng_set_launch(ctx, 4)
        kw = dict(max_steps=steps, seed=SEED, trace=te, trace_stride=n)
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_EXP_CHAIN, n, st, **kw))
        runs = [_cols(te, cols)]
        e_mid = st.cpu().numpy().copy()
        b.brng_fill_base(ctx, b.BRNG_E)
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_EXP_CHAIN, n, st,
                                           flags=b.BRNG_FLAG_RESUME, **kw))
        runs.append(_cols(te, cols))
        cur = b.brng_get_cursors(ctx)
    finally:
        b.brng_destroy(ctx)
    for i, u in enumerate(units):
        sl = slice(64 * i, 64 * i + 64)
        starts = (e_first[sl], e_mid[64 * u:64 * u + 64])
        qcur = None
        for k, ge in enumerate(runs):
            e_in = np.vstack([starts[k][None, :], ge[:-1, sl]])
            q = oracle.expchain_replay(SEED, e_in, k == 0, cursors=qcur, unit0=u)
            qcur = q["cursors"]
            if k == 0:
                assert within(starts[0], q["e0"], q["e0tol"]).all(), u
            ok = within(ge[:, sl], q["etrace"], q["etol"])
            if not ok.all():
                t, c = np.argwhere(~ok)[0]
                print("expchain replay mismatch unit", u, "run", k, "step", t, "chain", c, "gpu",
                      ge[t, sl][c], "ref", q["etrace"][t, c], "tol", q["etol"][t, c], flush=True)
            assert ok.all(), (u, k)
        assert np.array_equal(cur[u], qcur[0]), u


def test_lda_full_size(dev):
    import torch
    b = _b()
    w = workloads.lda(n_docs=16384, sweeps=100, seed=SEED)
    nd, sweeps, W = w["n_docs"], w["sweeps"], 512
    off, ntok = w["offsets"], w["ntok"]
    total = int(off[-1])
    _say("lda full size", nd, sweeps, W)
    ctx = b.brng_create(SEED, nd, [W, W, W, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    th = torch.zeros((sweeps, total), dtype=torch.float32, device=dev)
    ct = torch.zeros((sweeps, total), dtype=torch.int32, device=dev)
    # two documents of each K, spread over the range
    docs = []
    for K in (8, 16, 64, 256):
        idx = np.nonzero(w["K"] == K)[0]
        docs += [int(idx[0]), int(idx[len(idx) // 2])]
    cols = [c for d in docs for c in range(off[d], off[d + 1])]
    try:
        b.brng_set_launch(ctx, 8)
        kw = dict(max_steps=sweeps, seed=SEED, trace=th, trace2=ct, trace_stride=total,
                  offsets=_t(off, dev), ntok=_t(ntok, dev))
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts, **kw))
        runs = [(_cols(th, cols), _cols(ct, cols))]
        for k in (b.BRNG_U, b.BRNG_N, b.BRNG_E):
            b.brng_fill_base(ctx, k)
        b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts,
                                           flags=b.BRNG_FLAG_RESUME, **kw))
        runs.append((_cols(th, cols), _cols(ct, cols)))
    finally:
        b.brng_destroy(ctx)
    diverged = 0
    pos = 0
    for d in docs:  # counts are integers: the resumed launch's start is exact
        K = int(off[d + 1] - off[d])
        o1 = np.array([0, K], dtype=np.int32)
        n1 = np.array([ntok[d]], dtype=np.int32)
        r1 = oracle.lda(SEED, o1, n1, sweeps, unit0=d)
        r2 = oracle.lda(SEED, o1, n1, sweeps, counts0=r1["counts"], cursors=r1["cursors"],
                        unit0=d)
        sl = slice(pos, pos + K)
        pos += K
        ok = True
        for (gth, gct), r in zip(runs, (r1, r2)):
            for s in range(sweeps):
                okt = within(gth[s, sl], r["theta"][s], r["theta_tol"][s]).all()
                okc = np.array_equal(gct[s, sl], r["ctrace"][s])
                if okt and okc:
                    continue
                if not okt:
                    assert r["gmargin"][s, 0] <= 1.0, (d, s)
                else:
                    assert r["mmargin"][s, 0] <= 0.0, (d, s)
                ok = False
                break
            if not ok:
                diverged += 1
                break
    print("lda full-size diverged docs", diverged, flush=True)
    assert diverged <= 1


@pytest.mark.parametrize("V", [4096, 50000])
def test_lda_full_full_size(dev, V):
    """Full LDA at the bench's size (16,384 documents, 64 topics, window
    512), over the bench's default vocabulary of 4,096 words (four blocks
    of 1,024 words per topic) and one of 50,000 (49 blocks): two calls of
    one sweep;
    every topic's phi and eight sampled documents (theta, every token's
    topic, n_d.) against the oracle replayed from the device's state, n_kw
    against the counts of the new assignment."""
    import torch
    b = _b()
    K, D = 64, 16384
    c = workloads.lda_corpus(n_docs=D, n_topics=K, n_vocab=V, seed=SEED)
    off, words, z0 = c["offsets"], c["words"], c["z0"]
    T = int(off[-1])
    U = b.brng_lda_full_units(K, V, D)
    du = U - D  # unit of document 0: the topic blocks come first
    _say("lda_full full size", D, K, V, T, "units", U)
    ctx = b.brng_create(SEED, U, [512, 512, 512, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    tz = _t(z0, dev)
    ndk = torch.zeros(D * K, dtype=torch.int32, device=dev)
    nkw = torch.zeros(K * V, dtype=torch.int32, device=dev)
    th = torch.zeros(D * K, dtype=torch.float32, device=dev)
    phi = torch.zeros(K * V, dtype=torch.float32, device=dev)
    docs = [0, 1, 777, 4096, 9000, 12345, 16000, D - 1]
    cur = oracle.new_cursors(U)
    z_in = z0.copy()
    flips = 0
    try:
        toff, tw = _t(off, dev), _t(words, dev)
        for call in range(2):
            b.brng_run_lda_full(ctx, K, V, 1, 0.1, 0.05, toff, tw, tz, ndk, nkw, th, phi)
            gz = tz.cpu().numpy()
            gth = th.cpu().numpy()
            gphi = np.ascontiguousarray(phi.cpu().numpy().reshape(V, K).T)
            gndk = ndk.cpu().numpy().reshape(D, K)
            gnkw = nkw.cpu().numpy().reshape(K, V)
            gcur = b.brng_get_cursors(ctx)
            torch.cuda.synchronize()
            r = oracle.lda_full_sweep(SEED, cur, K, V, 0.1, 0.05, off, words, z_in,
                                      theta32=gth, phi32=gphi.ravel(), docs=docs)
            okp = within(gphi, r["phi"], r["phi_tol"])
            bad_topics = [k for k in range(K) if not okp[k].all()]
            for k in bad_topics:
                assert r["phi_margin"][k] <= 1.0, (call, k)
            flips += len(bad_topics)
            for d in docs:
                okt = within(gth.reshape(D, K)[d], r["theta"][d], r["theta_tol"][d]).all()
                if not okt:
                    assert r["theta_margin"][d] <= 1.0, (call, d)
                    flips += 1
                sl = slice(off[d], off[d + 1])
                assert np.array_equal(gz[sl], r["z"][sl]), (call, d)
            ndk_ref, nkw_ref = oracle.lda_full_counts(K, V, off, words, gz)
            assert np.array_equal(gndk[docs], ndk_ref[docs]), call
            assert np.array_equal(gnkw, nkw_ref), call
            units = list(range(du)) + [du + d for d in docs]
            same = [u for u in units if np.array_equal(gcur[u], cur[u])]
            assert len(same) >= len(units) - 2, call
            cur[:] = gcur
            z_in = gz
    finally:
        b.brng_destroy(ctx)
    print("lda_full full-size flips", flips, flush=True)
    assert flips <= 2
