"""Pins of the oracle's binomial getter (the expanded library of Sec. 3's
future work): inversion against scipy's quantile function on the exact pool
uniforms, the law of Hormann's BTRD attempt enumerated over the uniform grid
against the binomial pmf, whole calls replayed from that enumeration,
chi-square, a randomized PIT over varying (n, p), consumption, edge cases."""
import numpy as np
import pytest
from scipy import special, stats

import oracle

KU = oracle.KIND_U
GRID = (2 * np.arange(2 ** 23, dtype=np.float64) + 1) * 2.0 ** -24


def _below(t):
    """P(g <= t) for g on the uniform grid."""
    return np.clip(np.floor((np.minimum(t, 2.0) * 2 ** 24 - 1) / 2) + 1, 0, 2 ** 23) / 2 ** 23


class Btrd:
    """Hormann's BTRD for p <= 1/2, tabulated (written from the method's
    description, independently of the oracle's C)."""

    def __init__(self, n, p):
        q = 1.0 - p
        self.n, self.p = n, p
        self.m = np.floor((n + 1) * p)
        spq = np.sqrt(n * p * q)
        self.b = 1.15 + 2.53 * spq
        self.a = -0.0873 + 0.0248 * self.b + 0.01 * p
        self.c = n * p + 0.5
        self.alpha = (2.83 + 5.1 / self.b) * spq
        self.vr = 0.92 - 4.2 / self.b
        self.urvr = 0.86 * self.vr
        self.lpm = stats.binom.logpmf(self.m, n, p)

    def k_of(self, U):
        us = 0.5 - np.abs(U)
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.floor((2 * self.a / us + self.b) * U + self.c), us

    def thr(self, k, us):
        """Accept iff V <= thr (V the scaled second variable)."""
        ok = (k >= 0) & (k <= self.n)
        kk = np.clip(k, 0, self.n)
        with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
            f = np.exp(stats.binom.logpmf(kk, self.n, self.p) - self.lpm)
            t = f * (self.a / (us * us) + self.b) / self.alpha
        return np.where(ok, t, -1.0), kk

    def law(self):
        n = self.n
        mass = np.zeros(int(n) + 1)
        # first uniform v <= u_r v_r: accepted at once
        v = GRID[GRID <= self.urvr]
        k, _ = self.k_of(v / self.vr - 0.43)
        ok = (k >= 0) & (k <= n)
        np.add.at(mass, k[ok].astype(np.int64), 1.0 / 2 ** 23)
        # u_r v_r < v < v_r: U from v, V = w v_r
        v = GRID[(GRID > self.urvr) & (GRID < self.vr)]
        U = v / self.vr - 0.93
        U = np.where(U >= 0, 0.5, -0.5) - U
        k, us = self.k_of(U)
        t, kk = self.thr(k, us)
        np.add.at(mass, kk.astype(np.int64), _below(t / self.vr) / 2 ** 23 * (t >= 0))
        # v >= v_r: U = w - 1/2, V = v
        k, us = self.k_of(GRID - 0.5)
        t, kk = self.thr(k, us)
        n_lt_vr = np.sum(GRID < self.vr)
        cnt = np.maximum(0.0, _below(np.minimum(t, 1.0)) * 2 ** 23 - n_lt_vr) * (t >= 0)
        np.add.at(mass, kk.astype(np.int64), cnt / 2 ** 46)
        return mass


def _draws(seed, n, p, calls):
    cur = oracle.new_cursors((len(n) + 63) // 64)
    out = [oracle.step_binomial(seed, cur, n, p)[0] for _ in range(calls)]
    return np.stack(out), cur


@pytest.mark.parametrize("n,p", [(5, 0.3), (40, 0.2), (19, 0.5), (7, 0.9), (1000, 0.997)])
def test_inversion_equals_quantile(n, p):
    """n min(p, 1-p) < 10: one uniform per draw, k = min{k : u <= F(k)} for
    p' = min(p, 1 - p), mirrored to n - k when p > 1/2."""
    N = 64 * 40
    k, cur = _draws(3, np.full(N, n), np.full(N, p), 1)
    assert np.all(cur[:, KU] == 64)
    u = np.concatenate([oracle.entries(3, q, KU, 0, 64) for q in range(N // 64)])
    pp = min(p, 1 - p)
    want = stats.binom.ppf(u, n, pp).astype(np.int64)
    near = np.abs(u - stats.binom.cdf(want, n, pp)) < 1e-12
    if p > 0.5:
        want = n - want
    assert near.sum() < 3
    assert np.array_equal(k[0][~near], want[~near])


@pytest.mark.parametrize("n,p", [(20, 0.5), (100, 0.3), (1000, 0.05), (100000, 0.4)])
def test_btrd_is_exact_by_enumeration(n, p):
    """The attempt's law over all grid uniforms is the binomial pmf to within
    the grid's discreteness (total variation < 2e-5), and the oracle's
    uniforms per draw match (1 + P(v > u_r v_r)) / P(accept)."""
    B = Btrd(n, p)
    mass = B.law()
    acc = mass.sum()
    law = mass / acc
    tv = 0.5 * np.abs(law - stats.binom.pmf(np.arange(n + 1), n, p)).sum()
    assert tv < 2e-5
    N = 64 * 256
    _, cur = _draws(29, np.full(N, n), np.full(N, p), 4)
    per_draw = cur[:, KU].sum() / (N * 4)
    per_attempt = 1.0 + np.mean(GRID > B.urvr)
    want = per_attempt / acc
    sd = 2.0 * np.sqrt(1 - acc) / acc / np.sqrt(N * 4) + 1e-3
    assert abs(per_draw - want) < 6 * sd


@pytest.mark.parametrize("n,p", [(60, 0.4), (5000, 0.02)])
def test_oracle_follows_the_attempts(n, p):
    """Whole calls on units whose slots share (n, p), replayed from the
    tabulated attempt: each round one uniform to every pending slot, then one
    more to every pending slot whose first uniform exceeded u_r v_r."""
    B = Btrd(n, p)
    N = 64 * 40
    cur = oracle.new_cursors(N // 64)
    out, _ = oracle.step_binomial(31, cur, np.full(N, n), np.full(N, p))
    compared = 0
    for q in range(N // 64):
        e = oracle.entries(31, q, KU, 0, 4096)
        pos, res, pend, close = 0, np.full(64, -1), np.ones(64, bool), False
        while pend.any():
            idx = np.nonzero(pend)[0]
            v = e[pos:pos + idx.size]
            pos += idx.size
            two = v > B.urvr
            w = np.zeros_like(v)
            w[two] = e[pos:pos + two.sum()]
            pos += int(two.sum())
            close |= bool(np.any(np.abs(v - B.urvr) < 1e-9) or np.any(np.abs(v - B.vr) < 1e-9))
            # immediate
            k1, _ = B.k_of(v / B.vr - 0.43)
            acc1 = ~two & (k1 >= 0) & (k1 <= n)
            # second uniform
            U = np.where(v >= B.vr, w - 0.5, 0.0)
            U2 = v / B.vr - 0.93
            U = np.where(v >= B.vr, U, np.where(U2 >= 0, 0.5, -0.5) - U2)
            V = np.where(v >= B.vr, v, w * B.vr)
            k2, us = B.k_of(U)
            t, kk = B.thr(k2, us)
            close |= bool(np.any(two & (np.abs(V - t) <= 1e-9 * np.maximum(1.0, np.abs(t)))))
            acc2 = two & (V <= t)
            kres = np.where(acc1, k1, kk)
            ok = acc1 | acc2
            res[idx[ok]] = kres[ok]
            pend[idx[ok]] = False
        if close:
            continue
        assert np.array_equal(out[64 * q:64 * q + 64], res), q
        assert cur[q, KU] == pos, q
        compared += 1
    assert compared >= 30


@pytest.mark.parametrize("n,p", [(30, 0.45), (400, 0.8), (10 ** 5, 0.01)])
def test_chi_square_against_pmf(n, p):
    N = 64 * 256
    k, _ = _draws(17, np.full(N, n), np.full(N, p), 6)
    k = k.ravel()
    lo, hi = stats.binom.ppf(1e-6, n, p), stats.binom.ppf(1 - 1e-6, n, p)
    edges = np.arange(lo, hi + 1)
    obs = np.array([np.sum(k == e) for e in edges])
    exp = stats.binom.pmf(edges, n, p) * k.size
    keep = exp >= 20
    o2 = np.concatenate([obs[keep], [k.size - obs[keep].sum()]])
    e2 = np.concatenate([exp[keep], [k.size - exp[keep].sum()]])
    chi = np.sum((o2 - e2) ** 2 / np.maximum(e2, 1e-9))
    assert stats.chi2.sf(chi, len(e2) - 1) > 1e-4


def test_varying_randomised_pit():
    rng = np.random.default_rng(6)
    N = 64 * 200
    n = np.exp(rng.uniform(0, np.log(1e5), N)).astype(np.int32)
    p = rng.uniform(size=N)
    k, _ = _draws(23, n, p, 4)
    v = rng.uniform(size=k.shape)
    pit = stats.binom.cdf(k - 1, n, p) + v * stats.binom.pmf(k, n, p)
    assert stats.kstest(pit.ravel(), "uniform").pvalue > 1e-3


def test_edges():
    n = np.array([0, 10, 10, -1, 10, 10, 7, 2 ** 30], dtype=np.int32)
    p = np.array([0.3, 0.0, 1.0, 0.5, -0.1, np.nan, 1.5, 0.5])
    cur = oracle.new_cursors(1)
    k, m = oracle.step_binomial(1, cur, n, p)
    assert list(k[:7]) == [0, 0, 10, -1, -1, -1, -1]
    assert abs(k[7] - 2 ** 29) < 6 * 2 ** 14
    assert np.all(np.isinf(m[3:7]))
    assert cur[0, KU] >= 4
