"""Pins of the oracle's conditional-binomial multinomial (the discrete
library of Sec. 3's future work): counts add up to n, the first component
is the binomial getter's call on the same stream, marginals and the joint
law against the multinomial pmf, and the edge cases."""
import numpy as np
from scipy import stats

import oracle

KU = oracle.KIND_U


def _items(K, n, w):
    off = np.concatenate([[0], np.cumsum(K)]).astype(np.int32)
    return off, np.asarray(n, dtype=np.int32), np.asarray(w, dtype=np.float64)


def test_sums_and_first_component_is_the_binomial_call():
    rng = np.random.default_rng(2)
    ni = 64 * 8
    K = rng.integers(2, 12, ni)
    n = rng.integers(0, 3000, ni)
    off, n, w = _items(K, n, rng.exponential(size=int(K.sum())))
    cur = oracle.new_cursors(8)
    x, _ = oracle.step_multinomial(7, cur, off, n, w)
    assert np.array_equal(np.add.reduceat(x, off[:-1]), n) and x.min() >= 0
    # component 0 is one binomial call over all items, first on the stream
    tot = np.add.reduceat(w, off[:-1])
    p0 = np.minimum(w[off[:-1]] / tot, 1.0)
    k0, _ = oracle.step_binomial(7, oracle.new_cursors(8), n, p0)
    assert np.array_equal(x[off[:-1]], k0)


def test_marginals_and_joint_law():
    ni = 64 * 256
    p = np.array([0.1, 0.2, 0.3, 0.4])
    n = 30
    off, nn, w = _items(np.full(ni, 4), np.full(ni, n), np.tile(p, ni))
    cur = oracle.new_cursors(ni // 64)
    xs = []
    for _ in range(3):
        x, _ = oracle.step_multinomial(11, cur, off, nn, w)
        xs.append(x.reshape(ni, 4))
    X = np.concatenate(xs)
    for k in range(4):
        obs = np.bincount(X[:, k], minlength=n + 1)
        exp = stats.binom.pmf(np.arange(n + 1), n, p[k]) * len(X)
        keep = exp >= 20
        chi = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
        assert stats.chi2.sf(chi, keep.sum() - 1) > 1e-4, k
    # joint law of (x0, x1, x2) on its most frequent cells
    keys, cnt = np.unique(X[:, :3], axis=0, return_counts=True)
    full = np.column_stack([keys, n - keys.sum(1)])
    pm = stats.multinomial.pmf(full, n, p) * len(X)
    keep = pm >= 20
    chi = np.sum((cnt[keep] - pm[keep]) ** 2 / pm[keep])
    assert stats.chi2.sf(chi, keep.sum() - 1) > 1e-4


def test_large_counts_use_btrd_and_keep_the_law():
    ni = 64 * 128
    p = np.array([0.5, 0.25, 0.15, 0.1])
    n = 100000
    off, nn, w = _items(np.full(ni, 4), np.full(ni, n), np.tile(p, ni))
    cur = oracle.new_cursors(ni // 64)
    x, _ = oracle.step_multinomial(13, cur, off, nn, w)
    X = x.reshape(ni, 4)
    for k in range(4):
        z = (X[:, k] - n * p[k]) / np.sqrt(n * p[k] * (1 - p[k]))
        assert abs(z.mean()) < 6 / np.sqrt(ni) and abs(z.std() - 1) < 0.05
    # the rejection path takes more than one uniform per draw on average
    assert cur[:, KU].sum() > 3 * ni


def test_edges():
    K = np.array([1, 3, 3, 3, 2, 0 + 2])
    n = np.array([17, 5, -1, 8, 9, 4])
    w = np.array([2.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, -1.0, 1.0, 0.0, 0.0, 0.0, np.nan])
    off, n, w = _items(K, n, w)
    cur = oracle.new_cursors(1)
    x, _ = oracle.step_multinomial(5, cur, off, n, w)
    assert x[0] == 17                                  # K = 1: everything, no draw
    assert x[1:4].sum() == 5 and x[1:4].min() >= 0
    assert list(x[4:7]) == [-1, -1, -1]                # n < 0
    assert list(x[7:10]) == [-1, -1, -1]               # a negative weight
    assert list(x[10:12]) == [0, 9]                    # zero weights: the last takes all
    assert list(x[12:14]) == [-1, -1]                  # a NaN weight
