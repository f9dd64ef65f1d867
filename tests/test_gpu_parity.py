"""GPU parity: the HIP library (through its C interface) against the oracle.

Every test prints the case it runs (seed, sizes, entry point) before the GPU
call, so a failing run names its case.
"""
import numpy as np
import pytest

import oracle
from paper_1412_4825_amd import workloads
from tests.parity_util import compare_rounds, compare_units, tol_of, within

pytestmark = pytest.mark.gpu

W_SMALL = [512, 512, 512, 512]


def _b():
    from paper_1412_4825_amd import binding
    return binding


def _say(*a):
    print("[case]", *a, flush=True)


def _ctx(seed, n, window, layout=0, prec=0):
    import torch
    b = _b()
    return b.brng_create(seed, n, window, layout=layout, prec=prec,
                         stream=torch.cuda.current_stream())


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


SEEDS = [0, 20141217, 0xFFFFFFFF00000005]


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_fill_base_windows(dev, seed, kind):
    b = _b()
    _say("fill_base", seed, kind)
    n = 130  # three units, the last one partial
    W = [1024] * 4
    ctx = _ctx(seed, n, W)
    try:
        for unit in range(3):
            base, ln, win = b.brng_get_window(ctx, kind, unit)
            assert base == 0 and ln == 1024
            ref = oracle.entries(seed, unit, kind, 0, 1024)
            if kind in (0, 3):
                assert np.array_equal(win.astype(np.float64), ref)
            else:
                assert within(win, ref, tol_of(ref)).all()
        # refill at a large cursor: block index above 2^32 exercises the
        # counter's high word
        cur = b.brng_get_cursors(ctx)
        big = (1 << 34) + 777
        cur[:, kind] = [big, big + 300, 5]
        b.brng_set_cursors(ctx, cur)
        b.brng_fill_base(ctx, kind)
        align = 128 if kind == 3 else 256
        for unit, c in enumerate([big, big + 300, 5]):
            base, ln, win = b.brng_get_window(ctx, kind, unit)
            assert base == c - c % align and ln == 1024
            ref = oracle.entries(seed, unit, kind, base, 1024)
            if kind in (0, 3):
                assert np.array_equal(win.astype(np.float64), ref)
            else:
                assert within(win, ref, tol_of(ref)).all()
    finally:
        b.brng_destroy(ctx)


def test_steps_reducible_and_gamma(dev):
    """Five calls of each one-at-a-time function (uniform, normal,
    exponential, Laplace, Weibull) with per-chain parameters, then gamma;
    small windows force refills inside the kernels; cursors bit-exact."""
    b = _b()
    n, seed = 1000, 99
    p = workloads.step_params(n, seed=5)
    _say("steps", n, seed)
    ctx = _ctx(seed, n, W_SMALL)
    cur = oracle.new_cursors((n + 63) // 64)
    out = _t(np.zeros(n, np.float32), dev)
    try:
        ta, tb = _t(p["a"], dev), _t(p["b"], dev)
        tmu, tsg, tl = _t(p["mu"], dev), _t(p["sigma"], dev), _t(p["lam"], dev)
        tal = _t(p["alpha"], dev)
        wk = np.exp(np.random.default_rng(3).uniform(np.log(0.2), np.log(20.0), n)).astype(np.float32)
        tk = _t(wk, dev)
        units = np.arange(n) // 64
        flips = set()
        for it in range(5):
            b.brng_step_uniform(ctx, ta, tb, out)
            r, tol = oracle.step_uniform(seed, cur, p["a"], p["b"])
            assert within(_np(out), r, tol).all()
            b.brng_step_normal(ctx, tmu, tsg, out)
            r, tol = oracle.step_normal(seed, cur, p["mu"], p["sigma"])
            assert within(_np(out), r, tol).all()
            b.brng_step_exp(ctx, tl, out)
            r, tol = oracle.step_exp(seed, cur, p["lam"])
            assert within(_np(out), r, tol).all()
            b.brng_step_laplace(ctx, tmu, tsg, out)
            r, tol = oracle.step_laplace(seed, cur, p["mu"], p["sigma"])
            assert within(_np(out), r, tol).all()
            b.brng_step_weibull(ctx, tl, tk, out)
            r, tol = oracle.step_weibull(seed, cur, p["lam"], wk)
            assert within(_np(out), r, tol).all()
        assert np.array_equal(b.brng_get_cursors(ctx), cur)
        gcur = cur.copy()
        b.brng_step_gamma(ctx, tal, out)
        g, tol, margin, nN, nE = oracle.step_gamma(seed, gcur, p["alpha"])
        bad, flips = compare_units(_np(out)[None], g[None], tol[None], margin[None], units)
        assert bad == 0
        got = b.brng_get_cursors(ctx)
        keep = np.array([u not in flips for u in range(got.shape[0])])
        assert np.array_equal(got[keep], gcur[keep])
        assert len(flips) <= 1
    finally:
        b.brng_destroy(ctx)


def test_step_uniform_fp64(dev):
    b = _b()
    n, seed = 300, 7
    _say("step_uniform fp64", n, seed)
    ctx = _ctx(seed, n, [0, 0, 0, 512], prec=1)
    rng = np.random.default_rng(1)
    a = rng.normal(size=n)
    bb = a + rng.exponential(size=n)
    out = _t(np.zeros(n), dev)
    cur = oracle.new_cursors(5)
    try:
        for it in range(6):
            b.brng_step_uniform(ctx, _t(a, dev), _t(bb, dev), out)
            r, _ = oracle.step_uniform(seed, cur, a, bb, kind=3)
            g = _np(out)
            assert np.all(np.abs(g - r) <= 4e-16 * np.maximum(np.abs(a), np.abs(r)) + 1e-300)
        assert np.array_equal(b.brng_get_cursors(ctx), cur)
    finally:
        b.brng_destroy(ctx)


def test_step_poisson(dev):
    """Poisson steps (inversion below 10, PTRS above) with per-chain rates
    spanning 1e-3..1e5 and the edge values (0, the switch at 10, invalid
    rates, 2^30); five calls through 512-entry windows; counts bit-exact,
    cursors bit-exact, flips only where the oracle's margin allows."""
    import torch
    b = _b()
    n, seed = 1000 + 17, 61
    rng = np.random.default_rng(8)
    lam = np.exp(rng.uniform(np.log(1e-3), np.log(1e5), n)).astype(np.float32)
    lam[:9] = [0.0, 9.999, 10.0, -1.0, np.nan, np.inf, 2.0 ** 30, 2.0 ** 31, 1e-30]
    _say("step_poisson", n, seed)
    ctx = _ctx(seed, n, W_SMALL)
    cur = oracle.new_cursors((n + 63) // 64)
    out = torch.zeros(n, dtype=torch.int32, device=dev)
    units = np.arange(n) // 64
    flipped = set()
    try:
        tl = _t(lam, dev)
        for it in range(5):
            b.brng_step_poisson(ctx, tl, out)
            k, margin = oracle.step_poisson(seed, cur, lam.astype(np.float64))
            g = _np(out)
            for u in np.unique(units[g != k]):
                if u in flipped:
                    continue
                sl = units == u
                assert margin[sl].min() <= 1.0, (it, u, g[sl], k[sl])
                flipped.add(int(u))
            ok = np.array([u not in flipped for u in units])
            assert np.array_equal(g[ok], k[ok])
        assert list(g[3:6]) == [-1, -1, -1] and g[7] == -1
        got = b.brng_get_cursors(ctx)
        keep = np.array([u not in flipped for u in range(got.shape[0])])
        assert np.array_equal(got[keep], cur[keep])
        assert len(flipped) <= 1
    finally:
        b.brng_destroy(ctx)


def test_step_binomial(dev):
    """Binomial steps (inversion when n min(p, 1-p) < 10, BTRD otherwise,
    mirrored above 1/2) with per-chain n up to 1e6 and p in [0, 1] plus the
    edge values; five calls through 512-entry windows; counts and cursors
    bit-exact, flips only where the oracle's margin allows."""
    import torch
    b = _b()
    m, seed = 1000 + 17, 62
    rng = np.random.default_rng(9)
    n = np.floor(np.exp(rng.uniform(0, np.log(1e6), m))).astype(np.int32)
    p = rng.uniform(size=m).astype(np.float32)
    n[:10] = [0, 10, 10, 40, -1, 10, 10, 10, 2 ** 30, 3]
    p[:10] = [0.3, 0.0, 1.0, 0.5, 0.5, -0.1, np.nan, 1.5, 0.5, 0.9999]
    _say("step_binomial", m, seed)
    ctx = _ctx(seed, m, W_SMALL)
    cur = oracle.new_cursors((m + 63) // 64)
    out = torch.zeros(m, dtype=torch.int32, device=dev)
    units = np.arange(m) // 64
    flipped = set()
    try:
        tn, tp = _t(n, dev), _t(p, dev)
        for it in range(5):
            b.brng_step_binomial(ctx, tn, tp, out)
            k, margin = oracle.step_binomial(seed, cur, n, p.astype(np.float64))
            g = _np(out)
            for u in np.unique(units[g != k]):
                if u in flipped:
                    continue
                sl = units == u
                assert margin[sl].min() <= 1.0, (it, u, g[sl], k[sl])
                flipped.add(int(u))
            ok = np.array([u not in flipped for u in units])
            assert np.array_equal(g[ok], k[ok])
        assert list(g[:3]) == [0, 0, 10] and list(g[4:8]) == [-1, -1, -1, -1]
        got = b.brng_get_cursors(ctx)
        keep = np.array([u not in flipped for u in range(got.shape[0])])
        assert np.array_equal(got[keep], cur[keep])
        assert len(flipped) <= 1
    finally:
        b.brng_destroy(ctx)


def test_step_multinomial(dev):
    """Conditional-binomial multinomial steps: 1,017 items with 1..40
    components (and one of 300), n up to 1e5, weights with zeros, and invalid
    items; five calls through 512-entry windows; counts and cursors
    bit-exact, flips only where the oracle's margin allows."""
    import torch
    b = _b()
    ni, seed = 1000 + 17, 63
    rng = np.random.default_rng(10)
    K = rng.integers(1, 41, ni)
    K[5] = 300
    n = np.floor(np.exp(rng.uniform(0, np.log(1e5), ni))).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(K)]).astype(np.int32)
    w = rng.exponential(size=int(off[-1])).astype(np.float32)
    w[rng.uniform(size=w.size) < 0.1] = 0.0
    n[7] = -1
    w[off[9]] = -1.0
    w[off[11]] = np.nan
    _say("step_multinomial", ni, seed)
    ctx = _ctx(seed, ni, W_SMALL)
    cur = oracle.new_cursors((ni + 63) // 64)
    out = torch.zeros(int(off[-1]), dtype=torch.int32, device=dev)
    unit_of_comp = np.repeat(np.arange(ni) // 64, K)
    units = np.arange(ni) // 64
    flipped = set()
    try:
        toff, tn, tw = _t(off, dev), _t(n, dev), _t(w, dev)
        for it in range(5):
            b.brng_step_multinomial(ctx, toff, tn, tw, out)
            x, margin = oracle.step_multinomial(seed, cur, off, n, w.astype(np.float64))
            g = _np(out)
            for u in np.unique(unit_of_comp[g != x]):
                if u in flipped:
                    continue
                assert margin[units == u].min() <= 1.0, (it, u)
                flipped.add(int(u))
            ok = np.array([u not in flipped for u in unit_of_comp])
            assert np.array_equal(g[ok], x[ok])
        sums = np.add.reduceat(g, off[:-1])
        good = np.array([i not in (7, 9, 11) for i in range(ni)])
        assert np.array_equal(sums[good], n[good])
        assert np.all(g[off[7]:off[8]] == -1)
        got = b.brng_get_cursors(ctx)
        keep = np.array([u not in flipped for u in range(got.shape[0])])
        assert np.array_equal(got[keep], cur[keep])
        assert len(flipped) <= 1
    finally:
        b.brng_destroy(ctx)


def test_step_dirichlet_ragged(dev):
    b = _b()
    it = workloads.dirichlet_items(150, kmin=1, kmax=300, seed=3)
    seed = 1234
    n = it["K"].size
    _say("step_dirichlet", n, seed)
    ctx = _ctx(seed, n, W_SMALL, layout=1)
    out = _t(np.zeros(it["alpha"].size, np.float32), dev)
    cur = oracle.new_cursors(n)
    try:
        for rep in range(2):
            b.brng_step_dirichlet(ctx, _t(it["offsets"], dev), _t(it["alpha"], dev), out)
            th, tol, margin = oracle.step_dirichlet(seed, cur, it["offsets"], it["alpha"])
            g = _np(out)
            ok = within(g, th, tol)
            bad_items = [i for i in range(n) if not ok[it["offsets"][i]:it["offsets"][i + 1]].all()]
            assert all(margin[i] <= 1.0 for i in bad_items)
            assert len(bad_items) <= 1
        got = b.brng_get_cursors(ctx)
        assert (got == cur).all(axis=1).sum() >= n - 1
    finally:
        b.brng_destroy(ctx)


def _first_entries(ctx, kind, n):
    """The first entries of every unit's window of `kind` as the library
    holds them (fp32), read right after brng_create filled the windows from
    cursor 0: the starting state a fresh chain run draws with its first
    call (lane c of unit u takes entry c)."""
    b = _b()
    out = np.zeros(n, dtype=np.float32)
    for u in range((n + 63) // 64):
        base, ln, win = b.brng_get_window(ctx, kind, u)
        assert base == 0 and ln >= 64
        k = min(64, n - 64 * u)
        out[64 * u:64 * u + k] = win[:k]
    return out


def _gibbs(ctx, model, n, state, max_steps, seed, dev, trace=None, trace2=None, stride=0, **kw):
    b = _b()
    d = b.gibbs_desc(model, n, state, max_steps=max_steps, seed=seed, trace=trace, trace2=trace2,
                     trace_stride=stride, **kw)
    b.brng_run_gibbs(ctx, d)


def test_triangle_full_size_bit_exact(dev):
    """1,024 chains x 10,000 iterations in fp64 (the paper's example at the
    configured size): every x and y of every iteration, bit for bit."""
    import torch
    b = _b()
    n, iters, seed = 1024, 10000, 20141217
    _say("triangle", n, iters, seed)
    ctx = _ctx(seed, n, [0, 0, 0, 4096])
    st = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    tx = torch.zeros((iters, n), dtype=torch.float64, device=dev)
    ty = torch.zeros((iters, n), dtype=torch.float64, device=dev)
    try:
        _gibbs(ctx, b.BRNG_MODEL_TRIANGLE_F64, n, st, iters, seed, dev, tx, ty, n)
        r = oracle.triangle(seed, n, iters)
        assert np.array_equal(_np(tx), r["xtrace"])
        assert np.array_equal(_np(ty), r["ytrace"])
        s = _np(st)
        assert np.array_equal(s[:n], r["x"]) and np.array_equal(s[n:], r["y"])
        assert np.array_equal(b.brng_get_cursors(ctx), r["cursors"])
    finally:
        b.brng_destroy(ctx)


NORMEXP_WINDOWS = [[512, 512, 512, 512], [0, 4096, 4096, 0], [0, 65536, 65536, 0]]


@pytest.mark.parametrize("window", NORMEXP_WINDOWS)
def test_normexp_chains(dev, window):
    """Windows below 2,304 entries take the general (ballot) path, larger
    ones the pipelined full-wave path; both must match the oracle."""
    import torch
    b = _b()
    n, steps, seed = 2048 + 40, 301, 5
    _say("normexp", n, steps, seed, window)
    ctx = _ctx(seed, n, window)
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    te = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    try:
        s_first = _first_entries(ctx, b.BRNG_N, n)
        _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n, st, steps, seed, dev, ts, te, n)
        gs, ge = _np(ts), _np(te)
        gcur = b.brng_get_cursors(ctx)
        # the gate: every step replayed from the state the GPU held before
        # it, each output at the single-result bar
        q = oracle.normexp_replay(seed, np.vstack([s_first[None, :], gs[:-1]]), gs, True)
        assert within(s_first, q["s0"], q["s0tol"]).all()
        ok_s = within(gs, q["strace"], q["stol"])
        ok_e = within(ge, q["etrace"], q["etol"])
        print("normexp replay: s bad", int((~ok_s).sum()), "e bad", int((~ok_e).sum()), flush=True)
        assert ok_s.all() and ok_e.all()
        assert np.array_equal(gcur, q["cursors"])
        # free-running against the fp64 chain (bound propagated along it)
        r = oracle.normexp(seed, n, steps)
        assert within(gs, r["strace"], r["stol"]).all()
        assert within(ge, r["etrace"], r["etol"]).all()
        assert np.array_equal(gcur, r["cursors"])
    finally:
        b.brng_destroy(ctx)


def test_normexp_paths_bitwise_equal(dev):
    """The general and the pipelined path give the same bits, also when a
    run is resumed from the other path's cursors, and for an unaligned
    trace stride (scalar stores)."""
    import torch
    b = _b()
    n, seed = 64 * 20, 17
    outs = []
    for window, stride in (([0, 512, 512, 0], n), ([0, 2560, 2560, 0], n), ([0, 65536, 65536, 0], n + 1)):
        _say("normexp paths", window, stride)
        ctx = _ctx(seed, n, window)
        st = torch.zeros(n, dtype=torch.float32, device=dev)
        ts = torch.zeros((150, stride), dtype=torch.float32, device=dev)
        te = torch.zeros((150, stride), dtype=torch.float32, device=dev)
        try:
            _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n, st, 77, seed, dev, ts, te, stride)
            _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n, st, 73, seed, dev, ts[77:], te[77:], stride,
                   flags=b.BRNG_FLAG_RESUME)
            outs.append((_np(ts)[:, :n], _np(te)[:, :n], _np(st), b.brng_get_cursors(ctx)))
        finally:
            b.brng_destroy(ctx)
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("window", [[512, 512, 512, 512], [0, 0, 2560, 0]])
def test_expchain(dev, window):
    import torch
    b = _b()
    n, steps, seed = 640, 203, 8
    _say("expchain", n, steps, seed, window)
    ctx = _ctx(seed, n, window)
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    te = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    try:
        e_first = _first_entries(ctx, b.BRNG_E, n)
        _gibbs(ctx, b.BRNG_MODEL_EXP_CHAIN, n, st, steps, seed, dev, te, None, n)
        ge = _np(te)
        gcur = b.brng_get_cursors(ctx)
        q = oracle.expchain_replay(seed, np.vstack([e_first[None, :], ge[:-1]]), True)
        assert within(e_first, q["e0"], q["e0tol"]).all()
        ok = within(ge, q["etrace"], q["etol"])
        print("expchain replay: bad", int((~ok).sum()), flush=True)
        assert ok.all()
        assert np.array_equal(gcur, q["cursors"])
        r = oracle.expchain(seed, n, steps)
        assert within(ge, r["etrace"], r["etol"]).all()
        assert np.array_equal(gcur, r["cursors"])
    finally:
        b.brng_destroy(ctx)


def _run_gamma_chain(dev, w, seed, window, perm=None):
    import torch
    b = _b()
    n = w["n_chains"]
    if perm is None:
        perm = b.brng_sort_by_length(w["steps"])
    smax = int(w["steps"].max())
    ctx = _ctx(seed, n, window)
    st = _t(w["alpha0"], dev)
    tg = torch.full((smax, n), float("nan"), dtype=torch.float32, device=dev)
    try:
        _gibbs(ctx, b.BRNG_MODEL_GAMMA_CHAIN, n, st, smax, seed, dev, tg, None, n,
               steps=_t(w["steps"], dev), perm=_t(perm, dev))
        return _np(tg), _np(st), b.brng_get_cursors(ctx), perm
    finally:
        b.brng_destroy(ctx)


def test_gamma_chains(dev):
    w = workloads.gamma_chain(n_chains=4096 + 17, lmin=5, lmax=120, seed=77)
    seed = 31
    _say("gamma_chain", w["n_chains"], seed)
    g, alpha, cur, perm = _run_gamma_chain(dev, w, seed, W_SMALL)
    assert np.array_equal(perm, oracle.sort_by_length(w["steps"]))
    units = np.arange(w["n_chains"]) // 64
    # the gate: every draw replayed from the shape the GPU formed for it
    # (0.1f + its previous draw), at the single-result bar
    shape = oracle.chain_shapes_fp32(w["alpha0"][perm], g)
    q = oracle.gamma_chain_replay(seed, shape, w["steps"], perm=perm)
    bad, flips = compare_rounds(g, q["gtrace"], q["gtol"], q["gmargin"], q["gr0"], q["gr1"], units)
    print("gamma replay flips", len(flips), "bad", bad, flush=True)
    assert bad == 0
    assert len(flips) <= 2
    keep = np.array([u not in flips for u in range(cur.shape[0])])
    assert np.array_equal(cur[keep], q["cursors"][keep])
    # free-running against the fp64 chain (shape bound propagated along it)
    r = oracle.gamma_chain(seed, w["alpha0"], w["steps"], perm=perm)
    bad, flips = compare_rounds(g, r["gtrace"], r["gtol"], r["gmargin"], r["gr0"], r["gr1"], units)
    print("gamma free-run flips", len(flips), "bad", bad, flush=True)
    assert bad == 0
    assert len(flips) <= 2


def test_gamma_trace_store_paths_bitwise_equal(dev):
    """Gamma-chain traces are the same bits whether rows go out one by one
    (a trace stride that is not a multiple of four) or four rows per 16-byte
    store (a stride that is), over a fresh launch of at most 37 steps per
    chain and a resumed launch of every chain's full length."""
    import torch
    b = _b()
    w = workloads.gamma_chain(n_chains=4096 + 17, lmin=20, lmax=300, seed=91)
    n, seed = w["n_chains"], 57
    perm = b.brng_sort_by_length(w["steps"])
    smax = int(w["steps"].max())
    outs = []
    for stride in (n, n + 3):  # n = 4,113: rows one by one; n + 3: four-row stores
        _say("gamma trace paths", n, stride)
        ctx = _ctx(seed, n, W_SMALL)
        st = _t(w["alpha0"], dev)
        tg = torch.full((smax, stride), float("nan"), dtype=torch.float32, device=dev)
        kw = dict(trace=tg, trace_stride=stride, perm=_t(perm, dev))
        try:
            _gibbs(ctx, b.BRNG_MODEL_GAMMA_CHAIN, n, st, 37, seed, dev, tg, None, stride,
                   steps=_t(np.minimum(w["steps"], 37).astype(np.int32), dev), perm=_t(perm, dev))
            _gibbs(ctx, b.BRNG_MODEL_GAMMA_CHAIN, n, st, smax, seed, dev, tg, None, stride,
                   steps=_t(w["steps"], dev), perm=_t(perm, dev), flags=b.BRNG_FLAG_RESUME)
            outs.append((_np(tg)[:, :n], _np(st), b.brng_get_cursors(ctx)))
        finally:
            b.brng_destroy(ctx)
    assert (n + 3) % 4 == 0 and n % 4 != 0
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y, equal_nan=True)


def test_gamma_unit_without_steps_leaves_its_columns_alone(dev):
    """A unit whose 64 chains all have zero steps (no lane holds a step when
    the launch starts) stores nothing: its trace columns stay as they were,
    its state and cursors do not move, and the other units' traces are the
    same bits as in a run where that unit has steps of its own.  Trace rows
    16-byte aligned (four-row stores) and not."""
    import torch
    b = _b()
    n, seed, smax = 3 * 64 + 5, 77, 90
    rng = np.random.default_rng(12)
    steps_b = rng.integers(20, smax + 1, size=n).astype(np.int32)
    steps_a = steps_b.copy()
    steps_a[64:128] = 0  # unit 1
    alpha0 = (0.1 * np.power(1000.0, rng.random(n))).astype(np.float32)
    for stride in (n + 3, n):
        outs = []
        for steps in (steps_a, steps_b):
            _say("gamma unit without steps", n, stride, int(steps[64:128].max()))
            ctx = _ctx(seed, n, W_SMALL)
            st = _t(alpha0, dev)
            tg = torch.full((smax, stride), float("nan"), dtype=torch.float32, device=dev)
            try:
                _gibbs(ctx, b.BRNG_MODEL_GAMMA_CHAIN, n, st, smax, seed, dev, tg, None, stride,
                       steps=_t(steps, dev))
                outs.append((_np(tg)[:, :n], _np(st), b.brng_get_cursors(ctx)))
            finally:
                b.brng_destroy(ctx)
        (ta, sa, ca), (tb, sb, cb) = outs
        other = np.r_[0:64, 128:n]
        assert np.array_equal(ta[:, other], tb[:, other], equal_nan=True)
        assert np.array_equal(sa[other], sb[other])
        assert np.isnan(ta[:, 64:128]).all()
        assert np.array_equal(sa[64:128], alpha0[64:128])
        assert np.array_equal(ca[[0, 2, 3]], cb[[0, 2, 3]])
        assert np.array_equal(ca[1], oracle.new_cursors(4)[1])


def test_lda(dev):
    import torch
    b = _b()
    w = workloads.lda(n_docs=240, sweeps=8, seed=5)
    seed = 404
    nd, total = w["n_docs"], int(w["offsets"][-1])
    _say("lda", nd, w["sweeps"], seed)
    ctx = _ctx(seed, nd, W_SMALL, layout=1)
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    th = torch.zeros((w["sweeps"], total), dtype=torch.float32, device=dev)
    ct = torch.zeros((w["sweeps"], total), dtype=torch.int32, device=dev)
    try:
        _gibbs(ctx, b.BRNG_MODEL_LDA, nd, counts, w["sweeps"], seed, dev, th, ct, total,
               offsets=_t(w["offsets"], dev), ntok=_t(w["ntok"], dev))
        r = oracle.lda(seed, w["offsets"], w["ntok"], w["sweeps"])
        diverged = _lda_diverged(_np(th), _np(ct), r, w["offsets"], w["sweeps"])
        print("lda diverged docs", diverged, flush=True)
        assert diverged <= 2
    finally:
        b.brng_destroy(ctx)


def _lda_diverged(gth, gct, r, off, sweeps):
    """Documents whose theta or counts left the oracle's, each at a decision
    within tolerance (asserted); the others match in every sweep."""
    diverged = 0
    for d in range(len(off) - 1):
        a, z = off[d], off[d + 1]
        for s in range(sweeps):
            okt = within(gth[s, a:z], r["theta"][s, a:z], r["theta_tol"][s, a:z]).all()
            okc = np.array_equal(gct[s, a:z], r["ctrace"][s, a:z])
            if okt and okc:
                continue
            # only a decision within tolerance may change the course
            if not okt:
                assert r["gmargin"][s, d] <= 1.0, (d, s)
            else:
                assert r["mmargin"][s, d] <= 0.0, (d, s)
            diverged += 1
            break
    return diverged


def test_lda_ragged_components_and_tokens(dev):
    """Component counts across the bin search's step boundaries (1, 2, 3,
    powers of two and their neighbours up to 256) and token counts at the
    edges of the two-calls-at-a-time token loop (0, 1, 63..65, 127..129,
    255..257), against the oracle."""
    import torch
    b = _b()
    Ks = [1, 2, 3, 4, 5, 7, 8, 9, 15, 17, 31, 33, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256]
    toks = [0, 1, 63, 64, 65, 127, 128, 129, 255, 256, 257, 200]
    K = np.array([Ks[i % len(Ks)] for i in range(2 * len(Ks))], dtype=np.int32)
    ntok = np.array([toks[i % len(toks)] for i in range(len(K))], dtype=np.int32)
    off = np.zeros(len(K) + 1, dtype=np.int32)
    off[1:] = np.cumsum(K)
    nd, total, sweeps, seed = len(K), int(off[-1]), 5, 909
    _say("lda ragged K", nd, sweeps, seed)
    ctx = _ctx(seed, nd, W_SMALL, layout=1)
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    th = torch.zeros((sweeps, total), dtype=torch.float32, device=dev)
    ct = torch.zeros((sweeps, total), dtype=torch.int32, device=dev)
    try:
        _gibbs(ctx, b.BRNG_MODEL_LDA, nd, counts, sweeps, seed, dev, th, ct, total,
               offsets=_t(off, dev), ntok=_t(ntok, dev))
        gct = _np(ct)
        r = oracle.lda(seed, off, ntok, sweeps)
        diverged = _lda_diverged(_np(th), gct, r, off, sweeps)
        # every sweep's counts add up to the document's tokens
        for d in range(nd):
            assert (gct[:, off[d]:off[d + 1]].sum(axis=1) == ntok[d]).all(), d
        print("lda ragged diverged docs", diverged, flush=True)
        assert diverged <= 2
    finally:
        b.brng_destroy(ctx)


def test_lda_document_order_invariance(dev):
    """Other windows and workgroup sizes (and an order hint, which the
    library ignores) give the same counts, traces and cursors bit for bit:
    each document is its own unit."""
    import torch
    b = _b()
    w = workloads.lda(n_docs=300, sweeps=6, seed=12)
    seed = 77
    nd, total, sw = w["n_docs"], int(w["offsets"][-1]), w["sweeps"]
    perms = [None, np.arange(nd, dtype=np.int32)[::-1].copy(),
             np.random.default_rng(4).permutation(nd).astype(np.int32)]
    # (document order, window, waves per workgroup); the bench's tuned shape
    # is the second
    cases = [(perms[0], 4096, 2), (perms[1], 512, 8), (perms[2], 1024, 4)]
    _say("lda order", nd, sw, seed)
    res = []
    for perm, win, wpb in cases:
        ctx = _ctx(seed, nd, [win] * 3 + [0], layout=1)
        counts = torch.zeros(total, dtype=torch.int32, device=dev)
        th = torch.zeros((sw, total), dtype=torch.float32, device=dev)
        ct = torch.zeros((sw, total), dtype=torch.int32, device=dev)
        tp = None if perm is None else _t(perm, dev)
        try:
            b.brng_set_launch(ctx, wpb)
            b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts, max_steps=sw,
                                               seed=seed, trace=th, trace2=ct, trace_stride=total,
                                               offsets=_t(w["offsets"], dev),
                                               ntok=_t(w["ntok"], dev), perm=tp))
            res.append((_np(counts), _np(th), _np(ct), b.brng_get_cursors(ctx)))
        finally:
            b.brng_destroy(ctx)
    for r in res[1:]:
        for x, y in zip(r, res[0]):
            assert np.array_equal(x, y)


def test_window_length_invariance(dev):
    """Window length is a speed knob only (Sec. 2.4): bitwise equal results."""
    w = workloads.gamma_chain(n_chains=1024 + 5, lmin=10, lmax=80, seed=9)
    outs = [_run_gamma_chain(dev, w, 3, [0, win, win, 0]) for win in (512, 768, 4096, 65536)]
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0], equal_nan=True)
        assert np.array_equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])


def test_step_api_equals_chain_kernel(dev):
    """A host loop of one-at-a-time calls (normal then exponential, the
    parameters computed between launches) follows the same streams as the
    normal/exponential chain kernel: s' bit for bit, e to 2 ulp (the loop
    forms 1 + s'^2 with two roundings, the kernel with one), same cursors."""
    import torch
    b = _b()
    n, steps, seed = 640, 40, 12
    _say("step loop vs chain", n, steps)
    ctx = _ctx(seed, n, W_SMALL)
    st = torch.zeros(n, dtype=torch.float32, device=dev)
    ts = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    te = torch.zeros((steps, n), dtype=torch.float32, device=dev)
    try:
        _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n, st, steps, seed, dev, ts, te, n)
        S, E, cur = _np(ts), _np(te), b.brng_get_cursors(ctx)
    finally:
        b.brng_destroy(ctx)
    ctx = _ctx(seed, n, W_SMALL)
    try:
        zeros = torch.zeros(n, dtype=torch.float32, device=dev)
        ones = torch.ones(n, dtype=torch.float32, device=dev)
        s = torch.zeros(n, dtype=torch.float32, device=dev)
        b.brng_step_normal(ctx, zeros, ones, s)  # s_0: the first Gaussian
        rs, re_ = [], []
        for t in range(steps):
            mu = s * 0.9
            sigma = s.abs() + 0.5
            sp = torch.empty_like(s)
            b.brng_step_normal(ctx, mu, sigma, sp)
            lam = sp * sp + 1.0
            e = torch.empty_like(s)
            b.brng_step_exp(ctx, lam, e)
            rs.append(sp)
            re_.append(e)
            s = sp
        assert np.array_equal(_np(torch.stack(rs)), S)
        ge = _np(torch.stack(re_)).astype(np.float64)
        assert np.all(np.abs(ge - E) <= 2 * np.spacing(np.abs(E).astype(np.float32)))
        assert np.array_equal(b.brng_get_cursors(ctx), cur)
    finally:
        b.brng_destroy(ctx)


def test_multi_request_equals_alone_and_resume(dev):
    """Two requests in one call give the same bits as each run alone; a run
    split in two with RESUME equals the straight run."""
    import torch
    b = _b()
    seed_a, seed_b = 41, 42
    n_a, n_b, steps = 700, 300, 120
    wa = workloads.gamma_chain(n_chains=n_a, lmin=20, lmax=steps, seed=4)
    perm_a = b.brng_sort_by_length(wa["steps"])

    def alone_gamma():
        g, al, cur, _ = _run_gamma_chain(dev, wa, seed_a, W_SMALL, perm=perm_a)
        return g, al

    def alone_normexp():
        ctx = _ctx(seed_b, n_b, W_SMALL)
        st = torch.zeros(n_b, dtype=torch.float32, device=dev)
        ts = torch.zeros((steps, n_b), dtype=torch.float32, device=dev)
        try:
            _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n_b, st, steps, seed_b, dev, ts, None, n_b)
            return _np(ts), _np(st)
        finally:
            b.brng_destroy(ctx)

    _say("multi-request")
    ga, ala = alone_gamma()
    sb, stb = alone_normexp()
    units_a = (n_a + 63) // 64
    ctx = _ctx(777, n_a + n_b + 64 * 3, W_SMALL)
    try:
        st_a = _t(wa["alpha0"], dev)
        tg = torch.full((steps, n_a), float("nan"), dtype=torch.float32, device=dev)
        st_b = torch.zeros(n_b, dtype=torch.float32, device=dev)
        ts = torch.zeros((steps, n_b), dtype=torch.float32, device=dev)
        d1 = b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n_a, st_a, max_steps=steps, seed=seed_a,
                          trace=tg, trace_stride=n_a, steps=_t(wa["steps"], dev),
                          perm=_t(perm_a, dev), unit_base=2)
        d2 = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, n_b, st_b, max_steps=steps, seed=seed_b,
                          trace=ts, trace_stride=n_b, unit_base=2 + units_a + 1)
        b.brng_run_gibbs(ctx, [d1, d2])
        assert np.array_equal(_np(tg), ga, equal_nan=True)
        assert np.array_equal(_np(st_a), ala)
        assert np.array_equal(_np(ts), sb)
        assert np.array_equal(_np(st_b), stb)
        # resume: 50 + 70 steps of the normexp request equal 120 straight
        st_c = torch.zeros(n_b, dtype=torch.float32, device=dev)
        t1 = torch.zeros((50, n_b), dtype=torch.float32, device=dev)
        t2 = torch.zeros((70, n_b), dtype=torch.float32, device=dev)
        _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n_b, st_c, 50, seed_b, dev, t1, None, n_b)
        _gibbs(ctx, b.BRNG_MODEL_NORMEXP, n_b, st_c, 70, seed_b, dev, t2, None, n_b,
               flags=b.BRNG_FLAG_RESUME)
        assert np.array_equal(np.vstack([_np(t1), _np(t2)]), sb)
        assert np.array_equal(_np(st_c), stb)
    finally:
        b.brng_destroy(ctx)


def _grid_words(seed, low_random=True):
    """All 2^23 uniform grid points (top 23 bits), random low 9 bits."""
    k = np.arange(1 << 23, dtype=np.uint64) << np.uint64(9)
    low = np.random.default_rng(seed).integers(0, 512, size=k.size, dtype=np.uint64)
    return (k | low).astype(np.uint32)


def _convert_gpu(dev, kind, words):
    import torch
    b = _b()
    n = words.size
    tw = _t(words.view(np.int32), dev)
    out = torch.zeros(n // 2 if kind == 3 else n, dtype=torch.float64 if kind == 3 else torch.float32,
                      device=dev)
    b.brng_convert(kind, tw, n, out, torch.cuda.current_stream())
    return _np(out)


def test_conversions_exhaustive_grid(dev):
    """Every uniform grid value through each conversion: U bit-exact; -ln U
    within the fp32 bar at every grid point; Box-Muller with each word of the
    pair running over the whole grid."""
    _say("convert grid")
    w = _grid_words(1)
    assert np.array_equal(_convert_gpu(dev, 0, w).astype(np.float64), oracle.convert(0, w))
    ref = oracle.convert(2, w)
    got = _convert_gpu(dev, 2, w)
    bad = ~within(got, ref, tol_of(ref))
    assert not bad.any(), (np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])
    rnd = np.random.default_rng(2).integers(0, 2**32, size=w.size, dtype=np.uint64).astype(np.uint32)
    for pair in (np.stack([w, rnd], 1).ravel(), np.stack([rnd, w], 1).ravel()):
        ref = oracle.convert(1, pair)
        got = _convert_gpu(dev, 1, pair)
        bad = ~within(got, ref, tol_of(ref))
        assert not bad.any(), (np.flatnonzero(bad)[:5], got[bad][:5], ref[bad][:5])
    pair = np.random.default_rng(3).integers(0, 2**32, size=1 << 22, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(_convert_gpu(dev, 3, pair), oracle.convert(3, pair))


def test_time_next_launch_brackets_the_chain_kernel(dev):
    """Events handed to brng_time_next_launch are recorded at the chain
    kernel's start and end: their interval is positive and lies inside the
    span of the call on the stream; the pair is used once (a second launch
    leaves the events as they were), and the results equal an untimed run."""
    import torch
    b = _b()
    w = workloads.gamma_chain(n_chains=4096, lmin=50, lmax=300, seed=3)
    n, smax, seed = w["n_chains"], int(w["steps"].max()), 31
    _say("timed chain launch", n, smax)
    outs = []
    for timed in (False, True):
        ctx = _ctx(seed, n, W_SMALL)
        st = _t(w["alpha0"], dev)
        tg = torch.zeros((smax, n), dtype=torch.float32, device=dev)
        try:
            kw = dict(max_steps=smax, seed=seed, trace=tg, trace_stride=n,
                      steps=_t(w["steps"], dev))
            if timed:
                k0 = torch.cuda.Event(enable_timing=True)
                k1 = torch.cuda.Event(enable_timing=True)
                s0 = torch.cuda.Event(enable_timing=True)
                s1 = torch.cuda.Event(enable_timing=True)
                b.brng_time_next_launch(ctx, k0, k1)
                s0.record()
            b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st, **kw))
            if timed:
                s1.record()
                torch.cuda.synchronize()
                kms, sms = k0.elapsed_time(k1), s0.elapsed_time(s1)
                print("kernel ms", kms, "span ms", sms, flush=True)
                assert 0.0 < kms <= sms * 1.001 + 1e-3
                outs.append((_np(tg), _np(st)))
                # used once: a second (resumed) launch does not move them
                b.brng_run_gibbs(ctx, b.gibbs_desc(b.BRNG_MODEL_GAMMA_CHAIN, n, st,
                                                   flags=b.BRNG_FLAG_RESUME, **kw))
                torch.cuda.synchronize()
                assert k0.elapsed_time(k1) == kms
                # a lone event is refused
                with pytest.raises(b.BrngError):
                    b.brng_time_next_launch(ctx, k0, None)
            else:
                outs.append((_np(tg), _np(st)))
        finally:
            b.brng_destroy(ctx)
    assert np.array_equal(outs[0][0], outs[1][0], equal_nan=True)
    assert np.array_equal(outs[0][1], outs[1][1])


def _lda_small_workload(seed):
    """Documents of 1..20 components (most at most 16, so that the plain
    launch packs them several to a wave) with token counts at the edges of a
    64-token call and of a 256-entry window chunk, plus Poisson(200)."""
    rng = np.random.default_rng(seed)
    nd = 301
    K = rng.integers(1, 17, nd).astype(np.int32)
    K[::13] = rng.integers(17, 21, K[::13].size)
    ntok = rng.poisson(200, nd).astype(np.int32)
    edge = [0, 1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 700]
    ntok[:len(edge)] = edge
    off = np.zeros(nd + 1, dtype=np.int32)
    off[1:] = np.cumsum(K)
    return off, ntok


def _lda_run(dev, off, ntok, sweeps, seed, batched, perm=None, flags=0, state=None):
    """One LDA request with traces and sums, alone (the plain launch, small
    documents packed) or beside a one-unit exponential-chain request (the
    batched launch, one document per wave).  Returns host copies of counts,
    traces, sums and the request's cursors."""
    import torch
    b = _b()
    nd, tot = len(off) - 1, int(off[-1])
    ctx = b.brng_create(seed, nd + 1, W_SMALL, layout=1, stream=torch.cuda.current_stream())
    try:
        counts = torch.zeros(tot, dtype=torch.int32, device=dev)
        th = torch.full((sweeps, tot), float("nan"), dtype=torch.float32, device=dev)
        ct = torch.full((sweeps, tot), -7, dtype=torch.int32, device=dev)
        sm = torch.zeros((2, tot), dtype=torch.float64, device=dev)
        keep = [_t(off, dev), _t(ntok, dev)]
        if perm is not None:
            keep.append(_t(perm, dev))
        d = b.gibbs_desc(b.BRNG_MODEL_LDA, nd, counts, max_steps=sweeps, seed=seed, trace=th,
                         trace2=ct, trace_stride=tot, offsets=keep[0], ntok=keep[1],
                         perm=keep[2] if perm is not None else None, sums=sm)
        descs = [d]
        if batched:
            e = torch.zeros(64, dtype=torch.float32, device=dev)
            keep.append(e)
            descs.append(b.gibbs_desc(b.BRNG_MODEL_EXP_CHAIN, 64, e, max_steps=3, seed=1,
                                      unit_base=nd))
        b.brng_run_gibbs(ctx, descs)
        first = [_np(th).copy(), _np(ct).copy()]
        # a second call resumes from the cursors and counts of the first
        descs[0].flags = b.BRNG_FLAG_RESUME
        b.brng_run_gibbs(ctx, descs)
        out = [_np(counts), _np(th), _np(ct), _np(sm)]
        out.append(b.brng_get_cursors(ctx)[:nd])
        return out + first
    finally:
        b.brng_destroy(ctx)


def test_lda_packed_documents_equal_one_per_wave(dev):
    """Documents with up to 16 components run several to a wave in the plain
    launch; every result (counts, theta and counts traces, sums, cursors,
    over a fresh and a resumed call) equals the batched launch's, which runs
    one document per wave, bit for bit; the theta of the packed run also
    passes the oracle."""
    off, ntok = _lda_small_workload(21)
    _say("lda packed vs one per wave", len(off) - 1)
    a = _lda_run(dev, off, ntok, 6, 77, batched=False)
    c = _lda_run(dev, off, ntok, 6, 77, batched=True)
    for i, (x, y) in enumerate(zip(a, c)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), i
    # the first call's six sweeps against the oracle
    r = oracle.lda(77, off, ntok, 6)
    diverged = _lda_diverged(a[5], a[6], r, off, 6)
    print("lda packed diverged docs", diverged, flush=True)
    assert diverged <= 2


def test_lda_document_order_checked_and_bad_documents_marked(dev):
    """An order with a repeated document is ignored (the results equal those
    of the index order); documents the kernels cannot serve (257
    components, a negative token count) get -1 in every count, the others
    are unaffected, in the plain and the batched launch."""
    off, ntok = _lda_small_workload(5)
    nd = len(off) - 1
    _say("lda bad order and bad documents", nd)
    ref = _lda_run(dev, off, ntok, 3, 9, batched=False)
    dup = np.arange(nd, dtype=np.int32)[::-1].copy()
    dup[3] = dup[4]
    got = _lda_run(dev, off, ntok, 3, 9, batched=False, perm=dup)
    for i, (x, y) in enumerate(zip(ref, got)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), i
    # a valid reversed order changes nothing either
    rev = np.arange(nd, dtype=np.int32)[::-1].copy()
    got = _lda_run(dev, off, ntok, 3, 9, batched=False, perm=rev)
    for i, (x, y) in enumerate(zip(ref, got)):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), i
    # bad documents: document 7 gets 257 components, document 11 -1 tokens
    K = np.diff(off).astype(np.int64)
    K[7] = 257
    off2 = np.zeros(nd + 1, dtype=np.int32)
    off2[1:] = np.cumsum(K)
    nt2 = ntok.copy()
    nt2[11] = -1
    for batched in (False, True):
        res = _lda_run(dev, off2, nt2, 3, 9, batched=batched)
        cnt = res[0]
        for dd in (7, 11):
            assert (cnt[off2[dd]:off2[dd + 1]] == -1).all(), (batched, dd)
        # every other document as in a run without the bad ones (its own
        # streams: the same results)
        good = [dd for dd in range(nd) if dd not in (7, 11)]
        for dd in good[:40]:
            a0, a1 = off2[dd], off2[dd + 1]
            r0, r1 = off[dd], off[dd + 1]
            assert np.array_equal(cnt[a0:a1], ref[0][r0:r1]), (batched, dd)
