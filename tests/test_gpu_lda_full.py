"""Full LDA (topic-word and document-topic Dirichlets, one topic per token)
against the oracle, through the C interface, one sweep per call and each
sweep replayed by the oracle from the device's own state:

- phi and theta within the fp32 bar of the oracle's fp64 draws, except rows
  that left it at a decision within tolerance (their unit then follows the
  device's cursors);
- every token's topic bit-exact given the device's fp32 theta and phi (the
  integer rule decides in the same precision on both sides);
- n_dk and n_kw equal to the counts of the new assignment;
- cursors equal for every unit without such a decision.

Cases: ragged documents (empty ones, up to a few hundred tokens) with a few
word ids outside the vocabulary, topic counts 1, 13 and 64 (the largest
whose weights a lane keeps in registers) and 65, 100, 256 and 1,024 (the
limit; weights formed from the row three times, with and without 16-byte
row loads),
vocabularies of 4,097, 8,192 and 30,000 words (five, eight and thirty
blocks of 1,024 words per topic, each block its own unit), a
launch of all sweeps at once equal to the sweep-by-sweep calls, and window
length and workgroup size changing nothing."""
import numpy as np
import pytest

import oracle
from paper_1412_4825_amd import workloads
from tests.parity_util import within

pytestmark = pytest.mark.gpu


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


def _corpus(D, K, V, mean_len, seed):
    c = workloads.lda_corpus(n_docs=D, n_topics=K, n_vocab=V, mean_len=mean_len, seed=seed)
    words = c["words"].copy()
    if words.size > 10:
        words[[3, words.size // 2]] = [V, -2]  # two words outside the vocabulary
    off = c["offsets"].copy()
    return off, words, c["z0"]


def _bufs(dev, D, K, V, words, z0):
    import torch
    return dict(words=_t(words, dev), z=_t(z0, dev),
                ndk=torch.zeros(D * K, dtype=torch.int32, device=dev),
                nkw=torch.zeros(K * V, dtype=torch.int32, device=dev),
                theta=torch.zeros(D * K, dtype=torch.float32, device=dev),
                phi=torch.zeros(K * V, dtype=torch.float32, device=dev))


@pytest.mark.parametrize("K,V,D,mean_len", [(13, 300, 40, 60.0), (64, 512, 24, 120.0),
                                            (1, 50, 10, 30.0), (64, 30000, 60, 150.0),
                                            (5, 4097, 20, 40.0), (3, 8192, 12, 50.0),
                                            (65, 300, 16, 60.0), (100, 200, 12, 80.0),
                                            (256, 120, 8, 60.0), (1024, 64, 6, 40.0)])
def test_lda_full_sweep_replay(dev, K, V, D, mean_len):
    import torch
    b = _b()
    seed, alpha, beta, sweeps = 777 + K, 0.1, 0.05, 4
    off, words, z0 = _corpus(D, K, V, mean_len, seed=K)
    U = b.brng_lda_full_units(K, V, D)
    nb = (U - D) // K  # vocabulary blocks per topic
    assert U == oracle.lda_full_units(K, V, D)
    _say("lda_full replay", K, V, D, int(off[-1]), "blocks", nb)
    ctx = b.brng_create(seed, U, [512, 512, 512, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    buf = _bufs(dev, D, K, V, words, z0)
    toff = _t(off, dev)
    cur = oracle.new_cursors(U)
    z_in = z0.copy()
    flips = 0
    try:
        for s in range(sweeps):
            b.brng_run_lda_full(ctx, K, V, 1, alpha, beta, toff, buf["words"], buf["z"],
                                buf["ndk"], buf["nkw"], buf["theta"], buf["phi"])
            gz, gth = _np(buf["z"]), _np(buf["theta"])
            gphi = np.ascontiguousarray(_np(buf["phi"]).reshape(V, K).T)  # word-major on device
            gndk, gnkw = _np(buf["ndk"]), _np(buf["nkw"])
            gcur = b.brng_get_cursors(ctx)[:U]
            r = oracle.lda_full_sweep(seed, cur, K, V, alpha, beta, off, words, z_in,
                                      theta32=gth, phi32=gphi.ravel())
            flipped = set()
            okp = within(gphi.reshape(K, V), r["phi"], r["phi_tol"])
            for k in range(K):
                if not okp[k].all():
                    assert r["phi_margin"][k] <= 1.0, ("phi", s, k)
                    flipped.update(range(k * nb, (k + 1) * nb))  # the topic's blocks
            okt = within(gth.reshape(D, K), r["theta"], r["theta_tol"])
            for d in range(D):
                if not okt[d].all():
                    assert r["theta_margin"][d] <= 1.0, ("theta", s, d)
                    flipped.add(K * nb + d)
            flips += len(flipped)
            bad = np.nonzero(gz != r["z"])[0]
            if bad.size:
                i = bad[0]
                print("z mismatch sweep", s, "token", i, "gpu", gz[i], "ref", r["z"][i], flush=True)
            assert bad.size == 0, s
            assert np.array_equal(gndk.reshape(D, K), r["ndk"]), s
            assert np.array_equal(gnkw.reshape(K, V), r["nkw"]), s
            keep = np.array([u not in flipped for u in range(U)])
            assert np.array_equal(gcur[keep], cur[keep]), s
            cur[:] = gcur  # replay: follow the device from here
            z_in = gz
        print("lda_full flips", flips, flush=True)
        assert flips <= 2 * nb
    finally:
        b.brng_destroy(ctx)


def test_lda_full_many_sweeps_equal_single_sweeps(dev):
    """Six sweeps in one call equal six calls of one sweep, bit for bit, with
    or without the recount between calls, and the counts returned are those
    of the final assignment."""
    import torch
    b = _b()
    K, V, D, seed = 16, 256, 30, 4242
    off, words, z0 = _corpus(D, K, V, 80.0, seed=5)
    _say("lda_full sweeps in one call", K, V, D)
    res = []
    for calls, per, valid in ((1, 6, False), (6, 1, False), (6, 1, True)):
        ctx = b.brng_create(seed, K + D, [512, 512, 512, 0], layout=b.BRNG_LAYOUT_ITEMS,
                            stream=torch.cuda.current_stream())
        buf = _bufs(dev, D, K, V, words, z0)
        try:
            for c in range(calls):
                # with `valid`, calls after the first skip the recount
                b.brng_run_lda_full(ctx, K, V, per, 0.1, 0.05, _t(off, dev), buf["words"],
                                    buf["z"], buf["ndk"], buf["nkw"], buf["theta"], buf["phi"],
                                    counts_valid=valid and c > 0)
            res.append([_np(buf[k]) for k in ("z", "ndk", "nkw", "theta", "phi")] +
                       [b.brng_get_cursors(ctx)])
        finally:
            b.brng_destroy(ctx)
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert np.array_equal(x, y)
    ndk, nkw = oracle.lda_full_counts(K, V, off, words, res[0][0])
    assert np.array_equal(res[0][1].reshape(D, K), ndk)
    assert np.array_equal(res[0][2].reshape(K, V), nkw)


def test_lda_full_rejects_bad_arguments(dev):
    import torch
    b = _b()
    K, V, D = 4, 16, 3
    off, words, z0 = _corpus(D, K, V, 10.0, seed=1)
    ctx = b.brng_create(1, K + D, [512, 512, 512, 0], layout=b.BRNG_LAYOUT_ITEMS,
                        stream=torch.cuda.current_stream())
    buf = _bufs(dev, D, K, V, words, z0)
    try:
        for k, v, a in ((1025, V, 0.1), (K, (1 << 20) + 1, 0.1), (K, V, 0.0), (K + 1, V, 0.1),
                        (K, 4097, 0.1)):
            # K + 1 topics with D documents, or two vocabulary blocks per
            # topic, need more units than the context has
            with pytest.raises(b.BrngError):
                b.brng_run_lda_full(ctx, k, v, 1, a, 0.05, _t(off, dev), buf["words"], buf["z"],
                                    buf["ndk"], buf["nkw"], buf["theta"], buf["phi"])
    finally:
        b.brng_destroy(ctx)


@pytest.mark.parametrize("K,V,D", [(24, 700, 50), (8, 9000, 40), (100, 300, 30),
                                   (1024, 64, 12)])
def test_lda_full_window_and_launch_shape_invariance(dev, K, V, D):
    """Window length and waves per workgroup are speed knobs only: three
    configurations give the same topics, counts, draws and cursors bit for
    bit over three sweeps (also with three vocabulary blocks per topic, and
    at 1,024 topics, where eight waves per workgroup take 64 KiB of LDS)."""
    import torch
    b = _b()
    seed = 99
    off, words, z0 = _corpus(D, K, V, 90.0, seed=7)
    _say("lda_full window/launch invariance", K, V, D)
    res = []
    for win, wpb in ((512, 4), (4096, 1), (1024, 8)):
        ctx = b.brng_create(seed, b.brng_lda_full_units(K, V, D), [win, win, win, 0],
                            layout=b.BRNG_LAYOUT_ITEMS,
                            stream=torch.cuda.current_stream())
        buf = _bufs(dev, D, K, V, words, z0)
        try:
            b.brng_set_launch(ctx, wpb)
            b.brng_run_lda_full(ctx, K, V, 3, 0.1, 0.05, _t(off, dev), buf["words"], buf["z"],
                                buf["ndk"], buf["nkw"], buf["theta"], buf["phi"])
            res.append([_np(buf[k]) for k in ("z", "ndk", "nkw", "theta", "phi")] +
                       [b.brng_get_cursors(ctx)])
        finally:
            b.brng_destroy(ctx)
    for r in res[1:]:
        for x, y in zip(res[0], r):
            assert np.array_equal(x, y)
