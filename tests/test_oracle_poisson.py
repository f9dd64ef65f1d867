"""Pins of the oracle's Poisson getter (the expanded library of Sec. 3's
future work): inversion against scipy's quantile function on the exact pool
uniforms, chi-square of the transformed-rejection path against the Poisson
pmf, a randomized PIT over varying lambda, consumption and edge cases."""
import numpy as np
import pytest
from scipy import stats

import oracle

KU = oracle.KIND_U


def _draws(seed, lam_per_chain, calls):
    lam = np.asarray(lam_per_chain, dtype=np.float64)
    cur = oracle.new_cursors((lam.size + 63) // 64)
    out = [oracle.step_poisson(seed, cur, lam)[0] for _ in range(calls)]
    return np.stack(out), cur


@pytest.mark.parametrize("lam", [0.01, 0.7, 3.0, 9.99])
def test_inversion_equals_quantile(lam):
    """Below 10 each draw is min{k : u <= F(k)} of its own uniform: one call
    gives chain c of unit q the entry c - 64 q of the unit's U pool."""
    n = 64 * 40
    k, cur = _draws(3, np.full(n, lam), 1)
    assert np.all(cur[:, KU] == 64)
    u = np.concatenate([oracle.entries(3, q, KU, 0, 64) for q in range(n // 64)])
    want = stats.poisson.ppf(u, lam).astype(np.int64)
    # scipy evaluates the cdf its own way: skip uniforms within 1e-12 of it
    near = np.abs(u - stats.poisson.cdf(want, lam)) < 1e-12
    assert near.sum() < 3
    assert np.array_equal(k[0][~near], want[~near])


@pytest.mark.parametrize("lam", [0.5, 3.0, 9.9, 10.0, 37.0, 1000.0])
def test_chi_square_against_pmf(lam):
    n = 64 * 256
    k, _ = _draws(17, np.full(n, lam), 8)
    k = k.ravel()
    assert k.min() >= 0
    lo, hi = stats.poisson.ppf(1e-6, lam), stats.poisson.ppf(1 - 1e-6, lam)
    edges = np.arange(lo, hi + 2)
    obs = np.array([np.sum(k < lo)] + [np.sum(k == e) for e in edges[:-1]] + [np.sum(k > hi)])
    p = np.concatenate([[stats.poisson.cdf(lo - 1, lam)], stats.poisson.pmf(edges[:-1], lam),
                        [stats.poisson.sf(hi, lam)]])
    exp = p * k.size
    # merge sparse bins
    keep = exp >= 20
    o2 = np.concatenate([obs[keep], [obs[~keep].sum()]])
    e2 = np.concatenate([exp[keep], [exp[~keep].sum()]])
    if e2[-1] < 20:
        o2, e2 = o2[:-1], e2[:-1]
        o2[-1] += obs[~keep].sum()
    chi = np.sum((o2 - e2) ** 2 / e2)
    assert stats.chi2.sf(chi, len(e2) - 1) > 1e-4
    assert abs(k.mean() - lam) < 6 * np.sqrt(lam / k.size)


def test_varying_lambda_randomised_pit():
    rng = np.random.default_rng(5)
    n = 64 * 200
    lam = np.exp(rng.uniform(np.log(0.01), np.log(1e4), n))
    k, _ = _draws(23, lam, 4)
    v = rng.uniform(size=k.shape)
    pit = stats.poisson.cdf(k - 1, lam) + v * stats.poisson.pmf(k, lam)
    assert stats.kstest(pit.ravel(), "uniform").pvalue > 1e-3


def test_consumption_and_edges():
    # small lambda: one uniform per draw; large: two per attempt
    _, cur = _draws(9, np.full(64 * 20, 50.0), 3)
    assert np.all(cur[:, KU] % 2 == 0)
    per_draw = cur[:, KU].sum() / (64 * 20 * 3)
    assert 2.0 <= per_draw < 2.8
    lam = np.array([0.0, -1.0, np.nan, np.inf, 2.0 ** 31, 2.0 ** 30, 5.0, 20.0])
    cur = oracle.new_cursors(1)
    k, m = oracle.step_poisson(1, cur, lam)
    assert list(k[:5]) == [0, -1, -1, -1, -1]
    assert abs(k[5] - 2.0 ** 30) < 8 * 2.0 ** 15 and k[6] >= 0 and k[7] >= 0
    assert np.all(np.isinf(m[1:5]))
    # lambda = 0 and 5 take one uniform each, 2^30 and 20 at least two
    assert cur[0, KU] >= 2 + 4


def _ptrs_tables(lam):
    """Hormann's PTRS for one attempt, tabulated over every uniform u of the
    pool grid ((2j + 1) 2^-24): the candidate k(u) and the probability that
    the second uniform v (same grid) accepts it."""
    from scipy import special
    j = np.arange(2 ** 23, dtype=np.float64)
    u = (2 * j + 1) * 2.0 ** -24
    b = 0.931 + 2.53 * np.sqrt(lam)
    a = -0.059 + 0.02483 * b
    invalpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2)
    U = u - 0.5
    us = 0.5 - np.abs(U)
    k = np.floor((2 * a / us + b) * U + lam + 0.43)
    kk = np.maximum(k, 0)
    with np.errstate(over="ignore", under="ignore"):
        vstar = np.exp(-lam + kk * np.log(lam) - special.gammaln(kk + 1)) * (a / (us * us) + b) / invalpha

    def below(t):  # P(v <= t) for v on the grid
        return np.clip(np.floor((np.minimum(t, 2.0) * 2 ** 24 - 1) / 2) + 1, 0, 2 ** 23) / 2 ** 23

    acc = np.where(us >= 0.07, below(np.maximum(vr, vstar)),
                   np.where(k < 0, 0.0, np.where(us < 0.013, below(np.minimum(us, vstar)), below(vstar))))
    return k, acc, vr, vstar, us


@pytest.mark.parametrize("lam", [10.0, 37.5, 1000.0])
def test_ptrs_is_exact_by_enumeration(lam):
    """The algorithm's output law, summed over all 2^23 grid uniforms and
    every second uniform, is the Poisson pmf to within the grid's
    discreteness (total variation < 2e-5; a wrong constant gives 1e-4 to
    1e-2); and the oracle's uniforms per draw match 2 / P(accept)."""
    k, acc, *_ = _ptrs_tables(lam)
    w = np.bincount(np.maximum(k, 0).astype(np.int64), weights=acc)
    pmf = w / w.sum()
    tv = 0.5 * np.abs(pmf - stats.poisson.pmf(np.arange(pmf.size), lam)).sum()
    assert tv < 2e-5
    p_acc = acc.mean()
    n = 64 * 256
    _, cur = _draws(29, np.full(n, lam), 4)
    per_draw = cur[:, KU].sum() / (n * 4)
    # attempts per draw are geometric: sd of the mean sqrt(1 - p) / p / sqrt(draws)
    sd = 2 * np.sqrt(1 - p_acc) / p_acc / np.sqrt(n * 4)
    assert abs(per_draw - 2 / p_acc) < 6 * sd


@pytest.mark.parametrize("lam", [12.0, 400.0])
def test_oracle_follows_the_attempts(lam):
    """Whole calls on units whose slots all have the same lambda, replayed
    from the enumerated attempt: each round, every pending slot takes u (in
    slot order), then v (in slot order), and is accepted iff v passes the
    attempt's tests, with value k(u).  Values and cursors must agree (units
    with a v within 1e-9 of its threshold are skipped)."""
    n = 64 * 48
    cur = oracle.new_cursors(n // 64)
    out, _ = oracle.step_poisson(31, cur, np.full(n, lam))
    k, acc, vr, vstar, us = _ptrs_tables(lam)
    thr = np.where(us >= 0.07, np.maximum(vr, vstar),
                   np.where(k < 0, -1.0, np.where(us < 0.013, np.minimum(us, vstar), vstar)))
    compared = 0
    for q in range(n // 64):
        e = oracle.entries(31, q, KU, 0, 4096)
        pos, res, pend, close = 0, np.full(64, -1), np.ones(64, bool), False
        while pend.any():
            idx = np.nonzero(pend)[0]
            u = e[pos:pos + idx.size]
            v = e[pos + idx.size:pos + 2 * idx.size]
            pos += 2 * idx.size
            j = np.round((u * 2 ** 24 - 1) / 2).astype(np.int64)
            t = thr[j]
            close |= bool(np.any(np.abs(v - t) <= 1e-9 * np.maximum(1.0, np.abs(t))))
            ok = v <= t
            res[idx[ok]] = k[j][ok]
            pend[idx[ok]] = False
        if close:
            continue
        assert np.array_equal(out[64 * q:64 * q + 64], res), q
        assert cur[q, KU] == pos, q
        compared += 1
    assert compared >= 40
