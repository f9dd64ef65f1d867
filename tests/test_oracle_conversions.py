"""Pins of the oracle's base deviates: the uniform grids (exhaustive), and the
exponential and Gaussian pools against their closed-form distributions.

The pools are the paper's buffers of reducible base distributions (Sec. 2.1,
Key Concepts: uniform, Gaussian, exponential, and the logarithm of uniform).
"""
import math

import numpy as np
from scipy import stats

import oracle

K_U, K_N, K_E, K_U64 = 0, 1, 2, 3


def test_u32_grid_exhaustive():
    """All 2^23 grid points (the top 23 bits of a word) with random low bits:
    values are strictly increasing with spacing exactly 2^-23, fill the open
    interval from 2^-24 to 1 - 2^-24, are symmetric about 1/2 and average
    exactly 1/2."""
    k = np.arange(1 << 23, dtype=np.uint64)
    low = np.random.default_rng(1).integers(0, 512, size=k.size, dtype=np.uint64)
    w = ((k << np.uint64(9)) | low).astype(np.uint32)
    u = oracle.u32_many(w)
    assert u[0] == 2.0 ** -24 and u[-1] == 1.0 - 2.0 ** -24
    d = np.diff(u)
    assert np.all(d == 2.0 ** -23)
    assert np.all(u + u[::-1] == 1.0)
    assert math.fsum(u) == 0.5 * u.size
    # every value is an fp32 number (24 significant bits at most)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_u32_ignores_low_bits():
    rng = np.random.default_rng(2)
    hi = rng.integers(0, 1 << 23, 1000, dtype=np.uint64) << np.uint64(9)
    for low in (0, 1, 255, 511):
        a = oracle.u32_many((hi | np.uint64(low)).astype(np.uint32))
        assert np.array_equal(a, oracle.u32_many(hi.astype(np.uint32)))


def test_u64_grid():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        wa, wb = (int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64))
        u = oracle.u64(wa, wb)
        assert 0.0 < u < 1.0
        m = u * 2.0 ** 53  # exact: u is (2k+1) 2^-53
        assert m == math.floor(m) and int(m) % 2 == 1
        k = (int(m) - 1) // 2
        assert k >> 20 == wa and (k & 0xFFFFF) == (wb >> 12)
    assert oracle.u64(0, 0) == 2.0 ** -53
    assert oracle.u64(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53


def test_entry_layout_matches_words():
    """Entry j of the uniform pool is word j % 4 of block j / 4."""
    w = oracle.words(77, 5, K_U, 10, 8)
    e = oracle.entries(77, 5, K_U, 40, 32)
    assert np.array_equal(e, oracle.u32_many(w))


def test_exponential_pool():
    e = np.concatenate([oracle.entries(9, u, K_E, 0, 100_000) for u in range(2)])
    assert e.min() > 0
    assert stats.kstest(e, "expon").pvalue > 1e-3
    assert abs(e.mean() - 1.0) < 5 / math.sqrt(e.size)
    # ln U = -E: the exponential pool is the paper's log-uniform buffer
    ulog = -e
    assert stats.kstest(np.exp(ulog), "uniform").pvalue > 1e-3


def test_gaussian_pool():
    z = np.concatenate([oracle.entries(9, u, K_N, 0, 100_000) for u in range(2)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    # Box-Muller structure: each pair's squared radius is Exp(mean 2), its
    # angle is uniform, and the two members are uncorrelated
    a, b = z[0::2], z[1::2]
    assert stats.kstest(a * a + b * b, "expon", args=(0, 2)).pvalue > 1e-3
    ang = (np.arctan2(b, a) / (2 * np.pi)) % 1.0
    assert stats.kstest(ang, "uniform").pvalue > 1e-3
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)


def test_pools_of_different_kinds_are_independent():
    u = oracle.entries(4, 0, K_U, 0, 50_000)
    e = oracle.entries(4, 0, K_E, 0, 50_000)
    # E is not a function of the same-index uniform (different counter word)
    assert abs(stats.spearmanr(u, e).statistic) < 5 / math.sqrt(u.size)


def test_convert_matches_pool_entries():
    """Converting a block's words by hand gives the pool entries."""
    for kind in (K_U, K_N, K_E, K_U64):
        w = oracle.words(321, 7, kind, 100, 64)
        per_block = 2 if kind == K_U64 else 4
        e = oracle.entries(321, 7, kind, 100 * per_block, 64 * per_block)
        assert np.array_equal(oracle.convert(kind, w), e)
