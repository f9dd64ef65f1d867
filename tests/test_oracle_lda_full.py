"""Pins of the oracle's full LDA sweep (topic-word and document-topic
Dirichlets, one categorical topic per token): the model's conditionals are
the plain definitions they are checked against.

- token rule: topic frequencies against p_k proportional to theta_k phi_k,w
  (chi-square), the extreme uniforms, a single admissible topic, all-zero
  weights and an invalid word;
- indexing: with replayed theta and phi that allow one topic per (document,
  word) pair, every token's topic is that one (a transposed phi or another
  document's theta fails);
- the Dirichlet shapes: over many sweeps from a fixed assignment the mean of
  phi_k,w is (beta + n_kw) / (V beta + n_k) and the mean of theta_d,k is
  (alpha + n_dk) / (K alpha + N_d);
- counts and cursors: counts add up to the tokens, each document's uniform
  cursor moves by its token count, topics take no uniforms.
"""
import numpy as np
import pytest
from scipy import stats

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _grid_u(rng, n):
    k = rng.integers(0, 1 << 23, size=n)
    return (2.0 * k + 1.0) / 16777216.0


def test_token_rule_frequencies_follow_theta_times_phi():
    rng = np.random.default_rng(5)
    K, V = 6, 4
    theta = rng.dirichlet(np.ones(K)).astype(np.float32)
    phi = rng.dirichlet(np.ones(V), size=K).astype(np.float32)
    w = 2
    p = theta.astype(np.float64) * phi[:, w]
    p /= p.sum()
    n = 30000
    z = np.array([oracle.lda_full_token_topic(theta, phi, w, u) for u in _grid_u(rng, n)])
    obs = np.bincount(z, minlength=K)
    chi = stats.chisquare(obs, p * n)
    assert chi.pvalue > 1e-3, (obs, p * n)


def test_token_rule_extremes_and_degenerate_weights():
    K, V = 5, 3
    theta = np.array([0.0, 0.25, 0.0, 0.5, 0.25], np.float32)
    phi = np.full((K, V), 1.0 / V, np.float32)
    lo, hi = 1.0 / 16777216.0, 1.0 - 1.0 / 16777216.0
    # the smallest uniform picks the first topic with weight, the largest the last
    assert oracle.lda_full_token_topic(theta, phi, 0, lo) == 1
    assert oracle.lda_full_token_topic(theta, phi, 0, hi) == 4
    # one admissible topic is always drawn
    one = np.zeros(K, np.float32)
    one[3] = 0.7
    rng = np.random.default_rng(1)
    assert {oracle.lda_full_token_topic(one, phi, 1, u) for u in _grid_u(rng, 200)} == {3}
    # all-zero weights: every topic equally likely
    zero = np.zeros(K, np.float32)
    z = [oracle.lda_full_token_topic(zero, phi, 2, u) for u in _grid_u(rng, 20000)]
    assert stats.chisquare(np.bincount(z, minlength=K)).pvalue > 1e-3
    # a word outside the vocabulary has no topic
    assert oracle.lda_full_token_topic(theta, phi, V, 0.5) == -1
    assert oracle.lda_full_token_topic(theta, phi, -1, 0.5) == -1


def _corpus(rng, D, V, lo, hi):
    off = np.zeros(D + 1, np.int32)
    off[1:] = np.cumsum(rng.integers(lo, hi + 1, size=D))
    words = rng.integers(0, V, size=int(off[-1])).astype(np.int32)
    return off, words


def test_each_token_uses_its_document_theta_and_its_word_phi():
    rng = np.random.default_rng(2)
    K, V, D = 7, 11, 9
    off, words = _corpus(rng, D, V, 1, 30)
    z0 = rng.integers(0, K, size=words.size).astype(np.int32)
    doc_of = np.repeat(np.arange(D), np.diff(off))
    # theta of document d one-hot at d mod K, phi open everywhere: the topic
    # is the document's
    theta = np.zeros((D, K), np.float32)
    theta[np.arange(D), np.arange(D) % K] = 1.0
    phi = np.full((K, V), 1.0 / V, np.float32)
    r = oracle.lda_full_sweep(3, oracle.new_cursors(K + D), K, V, 0.1, 0.05, off, words, z0,
                              theta32=theta.ravel(), phi32=phi.ravel())
    assert np.array_equal(r["z"], doc_of % K)
    # theta uniform, phi of word w open only at topic (3 w + 1) mod K: the
    # topic is the word's (a transposed phi, V != K, could not give this)
    theta = np.full((D, K), 1.0 / K, np.float32)
    phi = np.zeros((K, V), np.float32)
    phi[(3 * np.arange(V) + 1) % K, np.arange(V)] = 1.0
    r = oracle.lda_full_sweep(3, oracle.new_cursors(K + D), K, V, 0.1, 0.05, off, words, z0,
                              theta32=theta.ravel(), phi32=phi.ravel())
    assert np.array_equal(r["z"], (3 * words + 1) % K)


def test_counts_and_cursors():
    rng = np.random.default_rng(3)
    K, V, D = 5, 40, 12
    off, words = _corpus(rng, D, V, 0, 60)
    words[3] = V  # one invalid word
    z0 = rng.integers(0, K, size=words.size).astype(np.int32)
    cur = oracle.new_cursors(K + D)
    before = cur.copy()
    r = oracle.lda_full_sweep(11, cur, K, V, 0.2, 0.01, off, words, z0)
    ntok = np.diff(off)
    valid = np.array([0 <= w < V for w in words])
    assert r["z"][3] == -1
    assert (r["z"][valid] >= 0).all() and (r["z"][valid] < K).all()
    per_doc_valid = np.array([valid[off[d]:off[d + 1]].sum() for d in range(D)])
    assert np.array_equal(r["ndk"].sum(axis=1), per_doc_valid)
    assert r["nkw"].sum() == valid.sum()
    assert np.array_equal(r["ndk"].sum(axis=0), r["nkw"].sum(axis=1))
    # documents take one uniform per token, topics none
    assert np.array_equal(cur[K:, oracle.KIND_U] - before[K:, oracle.KIND_U], ntok.astype(np.uint64))
    assert np.array_equal(cur[:K, oracle.KIND_U], before[:K, oracle.KIND_U])
    # every unit drew its Dirichlet from N and E
    assert (cur[:, oracle.KIND_N] > before[:, oracle.KIND_N]).all()
    assert (cur[:, oracle.KIND_E] > before[:, oracle.KIND_E]).all()
    # phi and theta rows are distributions
    assert np.allclose(r["phi"].sum(axis=1), 1.0)
    assert np.allclose(r["theta"].sum(axis=1), 1.0)


@pytest.mark.parametrize("vblock", [oracle.LDA_FULL_VBLOCK, 4])
def test_dirichlet_shapes_are_prior_plus_counts(vblock):
    """With vblock 4 each topic's six words are two blocks of two units: the
    means still follow the whole topic's counts."""
    rng = np.random.default_rng(4)
    K, V, D = 3, 6, 4
    alpha, beta = 0.3, 0.2
    off, words = _corpus(rng, D, V, 15, 25)
    z0 = rng.integers(0, K, size=words.size).astype(np.int32)
    ndk, nkw = oracle.lda_full_counts(K, V, off, words, z0)
    cur = oracle.new_cursors(oracle.lda_full_units(K, V, D, vblock))
    n = 3000
    phis = np.zeros((n, K, V))
    ths = np.zeros((n, D, K))
    for s in range(n):
        # the assignment is reset each time: the shapes stay beta + n_kw and
        # alpha + n_dk while the cursors move on
        r = oracle.lda_full_sweep(17, cur, K, V, alpha, beta, off, words, z0, vblock=vblock)
        phis[s], ths[s] = r["phi"], r["theta"]
    m_phi = (beta + nkw) / (V * beta + nkw.sum(axis=1, keepdims=True))
    m_th = (alpha + ndk) / (K * alpha + ndk.sum(axis=1, keepdims=True))
    # Dirichlet marginal variances give the standard error of the mean
    a0 = V * beta + nkw.sum(axis=1, keepdims=True)
    se_phi = np.sqrt(m_phi * (1 - m_phi) / (a0 + 1) / n)
    b0 = K * alpha + ndk.sum(axis=1, keepdims=True)
    se_th = np.sqrt(m_th * (1 - m_th) / (b0 + 1) / n)
    assert (np.abs(phis.mean(axis=0) - m_phi) < 5 * se_phi + 1e-12).all()
    assert (np.abs(ths.mean(axis=0) - m_th) < 5 * se_th + 1e-12).all()


def test_document_subset_equals_full_sweep_on_those_documents():
    rng = np.random.default_rng(6)
    K, V, D = 6, 30, 10
    off, words = _corpus(rng, D, V, 0, 40)
    z0 = rng.integers(0, K, size=words.size).astype(np.int32)
    full = oracle.lda_full_sweep(8, oracle.new_cursors(K + D), K, V, 0.1, 0.05, off, words, z0)
    docs = [1, 4, 9]
    cur = oracle.new_cursors(K + D)
    sub = oracle.lda_full_sweep(8, cur, K, V, 0.1, 0.05, off, words, z0, docs=docs)
    assert np.array_equal(sub["phi"], full["phi"])
    for d in docs:
        assert np.array_equal(sub["theta"][d], full["theta"][d])
        sl = slice(off[d], off[d + 1])
        assert np.array_equal(sub["z"][sl], full["z"][sl])
        assert np.array_equal(cur[K + d], full["cursors"][K + d])
    others = [d for d in range(D) if d not in docs]
    assert np.isnan(sub["theta"][others]).all()
    assert (cur[[K + d for d in others]] == 0).all()


def test_vocabulary_blocks_units_and_cursors():
    """Topics over a vocabulary of several blocks: topic k's block j is unit
    k nb + j and document d unit K nb + d; topic blocks take no uniforms and
    each draws its own N and E."""
    rng = np.random.default_rng(12)
    K, V, D, vb = 4, 23, 7, 5
    nb = -(-V // vb)
    assert oracle.lda_full_units(K, V, D, vb) == K * nb + D
    off, words = _corpus(rng, D, V, 5, 30)
    z0 = rng.integers(0, K, size=words.size).astype(np.int32)
    cur = oracle.new_cursors(K * nb + D)
    r = oracle.lda_full_sweep(31, cur, K, V, 0.1, 0.05, off, words, z0, vblock=vb)
    assert (cur[:K * nb, oracle.KIND_U] == 0).all()
    assert (cur[:, oracle.KIND_N] > 0).all() and (cur[:, oracle.KIND_E] > 0).all()
    assert np.allclose(r["phi"].sum(axis=1), 1.0)
    assert np.array_equal(cur[K * nb:, oracle.KIND_U], np.diff(off).astype(np.uint64))
    # document 3 is unit K nb + 3: its theta is that unit's Dirichlet over
    # alpha + n_3., and its tokens' topics take that unit's uniforms
    ndk0, _ = oracle.lda_full_counts(K, V, off, words, z0)
    d, du = 3, K * nb + 3
    sh = (np.float32(0.1) + ndk0[d].astype(np.float32)).astype(np.float32)
    x, _, _ = oracle.step_dirichlet(31, oracle.new_cursors(1), np.array([0, K], np.int32), sh,
                                    unit0=du)
    assert np.array_equal(r["theta"][d], x)
    a, b = int(off[d]), int(off[d + 1])
    u = oracle.entries(31, du, oracle.KIND_U, 0, b - a)
    phi32, th32 = r["phi"].astype(np.float32), r["theta"][d].astype(np.float32)
    zt = [oracle.lda_full_token_topic(th32, phi32, int(words[i]), u[i - a]) for i in range(a, b)]
    assert b > a and np.array_equal(r["z"][a:b], zt)
    # topic 2's block 1 (words 5..9) is unit 2 nb + 1: within the block the
    # ratios of phi are that unit's Dirichlet over beta + n_kw of those words
    _, nkw0 = oracle.lda_full_counts(K, V, off, words, z0)
    shapes = (np.float32(0.05) + nkw0[2, vb:2 * vb].astype(np.float32)).astype(np.float32)
    x, _, _ = oracle.step_dirichlet(31, oracle.new_cursors(1), np.array([0, vb], np.int32),
                                    shapes, unit0=2 * nb + 1)
    blk = r["phi"][2, vb:2 * vb]
    np.testing.assert_allclose(blk / blk.sum(), x, rtol=1e-12)
