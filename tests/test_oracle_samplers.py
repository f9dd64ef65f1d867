"""Pins of the oracle's varying-parameter samplers.

- Reducible transforms (Sec. 2.1): U(a,b), N(mu,sigma), Exp(lambda) with a
  different parameter per draw; pinned by probability integral transforms
  against scipy's closed-form CDFs.
- Gamma (the paper's GetGamma, Sec. 2.2; algorithm of Marsaglia & Tsang
  2000): PIT against the regularised incomplete gamma function, moments at
  fixed shapes, and the number of base deviates consumed per draw against
  the acceptance probability computed by quadrature (this ties the pool
  counters to the algorithm: a wrong term in the accept test changes it).
- Dirichlet from normalised gammas (Sec. 1, footnote): sums and Beta
  marginals.
- Multinomial from pool uniforms (integer rule): exact bin probabilities by
  enumerating every uniform on the grid, and a chi-square test.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle
from paper_1412_4825_amd import workloads

N = 20_000


def _cur(n, width=64):
    return oracle.new_cursors((n + width - 1) // width)


@pytest.fixture(scope="module")
def params():
    return workloads.step_params(N, seed=101)


def test_uniform_varying(params):
    a, b = params["a"].astype(np.float64), params["b"].astype(np.float64)
    out, tol = oracle.step_uniform(5, _cur(N), a, b)
    assert np.all(out > a) and np.all(out < b)
    assert stats.kstest((out - a) / (b - a), "uniform").pvalue > 1e-3
    assert np.all(tol > 0)


def test_normal_varying(params):
    mu, sg = params["mu"].astype(np.float64), params["sigma"].astype(np.float64)
    out, _ = oracle.step_normal(5, _cur(N), mu, sg)
    assert stats.kstest(special.ndtr((out - mu) / sg), "uniform").pvalue > 1e-3


def test_exponential_varying(params):
    lam = params["lam"].astype(np.float64)
    out, _ = oracle.step_exp(5, _cur(N), lam)
    assert stats.kstest(-np.expm1(-lam * out), "uniform").pvalue > 1e-3


def test_laplace_varying(params):
    """Laplace(mu, b) (GetLaplace, Sec. 2.2) with per-draw parameters: the
    PIT through the closed-form CDF is uniform."""
    mu = params["mu"].astype(np.float64)
    b = params["sigma"].astype(np.float64)
    out, _ = oracle.step_laplace(6, _cur(N), mu, b)
    assert stats.kstest(stats.laplace.cdf(out, loc=mu, scale=b), "uniform").pvalue > 1e-3


def test_laplace_takes_two_exponential_calls():
    """Two calls on the exponential pool, whole unit each: chain c's value is
    mu + b (E[c] - E[64 + c]) for a full unit; the partial unit likewise."""
    n = 100
    cur = _cur(n)
    out, _ = oracle.step_laplace(8, cur, np.zeros(n), np.ones(n))
    assert list(cur[:, 2]) == [128, 72]
    e0 = oracle.entries(8, 0, 2, 0, 128)
    e1 = oracle.entries(8, 1, 2, 0, 72)
    assert np.allclose(out[:64], e0[:64] - e0[64:], rtol=0, atol=1e-15)
    assert np.allclose(out[64:], e1[:36] - e1[36:], rtol=0, atol=1e-15)
    # symmetric about mu: as many draws on each side (binomial bounds)
    big, _ = oracle.step_laplace(9, _cur(N), np.full(N, 3.0), np.full(N, 2.0))
    k = int((big > 3.0).sum())
    assert abs(k - N / 2) < 5 * math.sqrt(N / 4)


def test_weibull_varying():
    """Weibull(lambda, k) (GetWeibull, Sec. 2.2) with per-draw scale and
    shape: the PIT through the closed-form CDF is uniform; the mean at a
    fixed shape is lambda Gamma(1 + 1/k)."""
    r = np.random.default_rng(11)
    lam = np.exp(r.uniform(np.log(0.01), np.log(100.0), N))
    k = np.exp(r.uniform(np.log(0.2), np.log(20.0), N))
    out, _ = oracle.step_weibull(6, _cur(N), lam, k)
    assert stats.kstest(stats.weibull_min.cdf(out, k, scale=lam), "uniform").pvalue > 1e-3
    out, _ = oracle.step_weibull(7, _cur(N), np.full(N, 2.0), np.full(N, 1.5))
    m, sd = 2.0 * special.gamma(1 + 1 / 1.5), 2.0 * math.sqrt(
        special.gamma(1 + 2 / 1.5) - special.gamma(1 + 1 / 1.5) ** 2)
    assert abs(out.mean() - m) < 5 * sd / math.sqrt(N)
    # shape 1 is the exponential of the same entries
    c1, c2 = _cur(N), _cur(N)
    w, _ = oracle.step_weibull(4, c1, np.full(N, 3.0), np.ones(N))
    e, _ = oracle.step_exp(4, c2, np.full(N, 1.0 / 3.0))
    assert np.allclose(w, e, rtol=1e-14, atol=0)


def test_calls_advance_cursors_in_slot_order():
    """Two calls over 100 chains: chain c of unit u takes entry (call * width
    + c - 64u) of its unit, for full units; the partial unit takes
    consecutive entries too."""
    n = 100
    cur = _cur(n)
    a, b = np.zeros(n), np.ones(n)
    o1, _ = oracle.step_uniform(3, cur, a, b)
    o2, _ = oracle.step_uniform(3, cur, a, b)
    assert list(cur[:, 0]) == [128, 72]
    e0 = oracle.entries(3, 0, 0, 0, 128)
    e1 = oracle.entries(3, 1, 0, 0, 72)
    assert np.array_equal(o1[:64], e0[:64]) and np.array_equal(o2[:64], e0[64:])
    assert np.array_equal(o1[64:], e1[:36]) and np.array_equal(o2[64:], e1[36:])


def test_gamma_pit_varying_shape(params):
    alpha = params["alpha"].astype(np.float64)
    g, tol, margin, nN, nE = oracle.step_gamma(8, _cur(N), alpha)
    assert np.all(g > 0)
    assert stats.kstest(special.gammainc(alpha, g), "uniform").pvalue > 1e-3
    assert np.all(nN >= 1)
    assert np.all(nE >= 1)
    # a boosted draw consumes one more exponential than its accept rounds
    assert np.all(nE[alpha < 1] >= 2)


@pytest.mark.parametrize("a", [0.1, 0.7, 1.0, 2.5, 30.0, 4600.0])
def test_gamma_fixed_shape(a):
    n = 20_000
    g, *_ = oracle.step_gamma(21, _cur(n), np.full(n, a))
    assert stats.kstest(g, "gamma", args=(a,)).pvalue > 1e-3
    se = math.sqrt(a / n)
    assert abs(g.mean() - a) < 5 * se
    # variance of a gamma sample mean-centred: a; se of s^2 ~ sqrt((kurt+2)/n) a
    assert abs(g.var() / a - 1.0) < 5 * math.sqrt((6.0 / a + 2.0) / n)


def _mt_acceptance(a):
    """P(one round accepts) and P(1 + c x > 0) for Marsaglia-Tsang at shape a
    by quadrature: a round accepts when 1 + c x > 0 and E > -d q(c x), and
    q <= 0, so P(accept | x) = exp(d q(c x))."""
    d = a - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)

    def q(y):
        return 3.0 * math.log1p(y) - 3.0 * y + 1.5 * y * y - y ** 3

    lo = -1.0 / c
    pacc = integrate.quad(lambda x: stats.norm.pdf(x) * math.exp(d * q(c * x)), lo, np.inf,
                          limit=200)[0]
    ppos = stats.norm.sf(lo)
    return pacc, ppos


@pytest.mark.parametrize("a", [1.0, 2.0, 10.0])
def test_gamma_consumption_matches_acceptance(a):
    n = 40_000
    g, tol, margin, nN, nE = oracle.step_gamma(31, _cur(n), np.full(n, a))
    pacc, ppos = _mt_acceptance(a)
    # rounds per draw are geometric with success pacc
    mean_rounds = 1.0 / pacc
    sd = math.sqrt((1 - pacc) / pacc ** 2 / n)
    assert abs(nN.mean() - mean_rounds) < 6 * sd + 1e-12
    # exponentials: one per round with 1 + c x > 0
    mean_e = ppos / pacc
    assert abs(nE.mean() - mean_e) < 6 * sd + 1e-12


def test_gamma_boost_consumption():
    n = 20_000
    g, tol, margin, nN, nE = oracle.step_gamma(32, _cur(n), np.full(n, 0.5))
    pacc, ppos = _mt_acceptance(1.5)
    assert abs((nE - 1).mean() - ppos / pacc) < 0.02


def test_gamma_invalid_shape_gives_nan_and_consumes_nothing():
    g, tol, margin, nN, nE = oracle.step_gamma(1, _cur(4), np.array([0.0, -1.0, np.nan, 2.0]))
    assert np.isnan(g[:3]).all() and g[3] > 0
    assert list(nN[:3]) == [0, 0, 0] and list(nE[:3]) == [0, 0, 0]


def test_dirichlet_sum_and_beta_marginals():
    av = np.array([0.3, 1.0, 2.5, 7.0, 0.1])
    K, items = av.size, 8000
    offsets = np.arange(items + 1, dtype=np.int32) * K
    alpha = np.tile(av, items)
    th, tol, m = oracle.step_dirichlet(12, oracle.new_cursors(items), offsets, alpha)
    th = th.reshape(items, K)
    assert np.all(np.abs(th.sum(axis=1) - 1.0) < 1e-12)
    a0 = av.sum()
    for k in range(K):
        assert stats.kstest(th[:, k], "beta", args=(av[k], a0 - av[k])).pvalue > 1e-3


def _rule_probabilities(theta):
    """Exact bin probabilities of the integer multinomial rule, by running the
    rule on every uniform of the 2^23-point grid."""
    q = np.rint(theta.astype(np.float32).astype(np.float64) * 2.0 ** 24).astype(np.int64)
    Q = int(q.sum())
    C = np.cumsum(q)
    j = np.arange(1 << 23, dtype=np.int64)
    t = (j * Q) >> 23
    bins = np.searchsorted(C, t, side="right")
    return np.bincount(bins, minlength=theta.size) / float(1 << 23), q, Q


def test_multinomial_rule_is_exact():
    theta = np.array([0.1, 0.2, 0.05, 0.6, 0.05])
    p, q, Q = _rule_probabilities(theta)
    # each bin's probability is its quantised weight to within one grid step
    assert np.all(np.abs(p - q / Q) <= 1.0 / (1 << 23) + 1e-15)
    assert np.all(np.abs(q / Q - theta) < 1e-6)


def test_multinomial_counts():
    theta = np.array([0.1, 0.2, 0.05, 0.6, 0.05])
    items, n = 4000, 200
    K = theta.size
    offsets = np.arange(items + 1, dtype=np.int32) * K
    ntok = np.full(items, n, np.int32)
    counts = oracle.multinomial(13, oracle.new_cursors(items), offsets, ntok, np.tile(theta, items))
    counts = counts.reshape(items, K)
    assert np.all(counts.sum(axis=1) == n) and np.all(counts >= 0)
    p, _, _ = _rule_probabilities(theta)
    tot = counts.sum(axis=0)
    chi2, pv = stats.chisquare(tot, f_exp=p * tot.sum())
    assert pv > 1e-3


def test_blocked_dirichlet_marginals_span_the_blocks():
    """A Dirichlet drawn in blocks of 3 components (each block from its own
    unit) is still Dirichlet(alpha) over all 8: the components sum to one and
    each follows Beta(alpha_k, A - alpha_k) with A the sum over every block
    (a normalisation within a block would put A_block there)."""
    av = np.array([0.3, 1.0, 2.5, 7.0, 0.1, 4.0, 0.7, 1.5])
    K, tb, draws = av.size, 3, 3000
    nb = -(-K // tb)
    cur = oracle.new_cursors(nb)
    th = np.zeros((draws, K))
    for i in range(draws):  # successive draws continue the blocks' streams
        th[i], _, _ = oracle.dirichlet_blocks(21, cur, av, tb, unit0=5)
    assert np.all(np.abs(th.sum(axis=1) - 1.0) < 1e-12)
    a0 = av.sum()
    for k in range(K):
        assert stats.kstest(th[:, k], "beta", args=(av[k], a0 - av[k])).pvalue > 1e-3, k


def test_blocked_dirichlet_block_streams():
    """Block j's gammas are those a single item of unit unit0 + j draws over
    that block's shapes: within a block the ratios of components equal the
    ratios of that item's draw, and each block's cursors move as that item's
    do.  With one block the draw is the single item's."""
    av = np.array([0.5, 2.0, 1.0, 3.0, 0.2, 6.0, 1.1])
    K, tb, unit0 = av.size, 3, 9
    nb = -(-K // tb)
    cur = oracle.new_cursors(nb)
    th, tol, m = oracle.dirichlet_blocks(4, cur, av, tb, unit0=unit0)
    assert m.shape == (nb,)
    for j in range(nb):
        lo, hi = j * tb, min(K, (j + 1) * tb)
        c1 = oracle.new_cursors(1)
        x, _, _ = oracle.step_dirichlet(4, c1, np.array([0, hi - lo], np.int32), av[lo:hi],
                                        unit0=unit0 + j)
        np.testing.assert_allclose(th[lo:hi] / th[lo:hi].sum(), x, rtol=1e-12)
        assert np.array_equal(cur[j], c1[0])
    # another unit's block would give other values
    c2 = oracle.new_cursors(1)
    x2, _, _ = oracle.step_dirichlet(4, c2, np.array([0, tb], np.int32), av[:tb], unit0=unit0 + 1)
    assert not np.allclose(th[:tb] / th[:tb].sum(), x2)
    # one block: the item's draw, with the same tolerances
    c3, c4 = oracle.new_cursors(1), oracle.new_cursors(1)
    a, ta, _ = oracle.dirichlet_blocks(4, c3, av, 64, unit0=unit0)
    b, tbb, _ = oracle.step_dirichlet(4, c4, np.array([0, K], np.int32), av, unit0=unit0)
    assert np.array_equal(a, b) and np.array_equal(ta, tbb) and np.array_equal(c3, c4)
