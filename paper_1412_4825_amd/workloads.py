"""Seeded synthetic workloads (inputs only; no sampler arithmetic lives here).

The paper measures on synthetic streams (Sec. 2.4: 200M samples per
distribution) and motivates the method with Gibbs sampling (Eq. 1, Fig. 1)
and LDA (Sec. 1).  These generators draw the inputs of the chain workloads
with numpy's PCG64 from a fixed workload seed; the same arrays feed the HIP
library and the CPU oracle.  Sizes can be scaled down for tests.
"""
from __future__ import annotations

import numpy as np

WORKLOAD_SEED = 20141217


def _rng(seed: int, salt: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, salt]))


def triangle(n_chains: int = 1024, iters: int = 10000):
    """Eq. 1 / Fig. 1: chains start at x = y = 0.5; nothing random here."""
    return dict(n_chains=n_chains, iters=iters)


def normexp(n_chains: int = 65536, steps: int = 1000):
    """s' ~ N(0.9 s, 0.5 + |s|), e ~ Exp(1 + s'^2); s_0 is the first Gaussian."""
    return dict(n_chains=n_chains, steps=steps)


def gamma_chain(n_chains: int = 262144, lmin: int = 50, lmax: int = 1000,
                seed: int = WORKLOAD_SEED):
    """Uneven lengths L ~ U{lmin..lmax}; alpha_0 = 0.1 * 1000^w, w ~ U(0,1)
    (log-uniform on [0.1, 100]), rounded to fp32."""
    r = _rng(seed, 3)
    steps = r.integers(lmin, lmax + 1, size=n_chains, dtype=np.int64).astype(np.int32)
    w = r.random(n_chains)
    alpha0 = (0.1 * np.power(1000.0, w)).astype(np.float32)
    return dict(n_chains=n_chains, steps=steps, alpha0=alpha0)


def lda(n_docs: int = 16384, sweeps: int = 100, mean_len: float = 200.0,
        ks=(8, 16, 64, 256), seed: int = WORKLOAD_SEED):
    """Documents with n_d ~ Poisson(mean_len) tokens and K_d drawn uniformly
    from `ks`; counts start at 0."""
    r = _rng(seed, 4)
    K = r.choice(np.asarray(ks, dtype=np.int64), size=n_docs).astype(np.int32)
    ntok = r.poisson(mean_len, size=n_docs).astype(np.int32)
    offsets = np.zeros(n_docs + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(K)
    return dict(n_docs=n_docs, sweeps=sweeps, K=K, ntok=ntok, offsets=offsets)


def lda_corpus(n_docs: int = 16384, n_topics: int = 64, n_vocab: int = 4096,
               mean_len: float = 200.0, seed: int = WORKLOAD_SEED):
    """A synthetic corpus drawn from the LDA generative model: topic-word
    distributions ~ Dir(0.05), document-topic ~ Dir(0.1), n_d ~
    Poisson(mean_len) tokens, each token's topic from its document and its
    word from that topic; the starting assignment is uniform over topics."""
    r = _rng(seed, 9)
    phi = r.dirichlet(np.full(n_vocab, 0.05), size=n_topics)
    theta = r.dirichlet(np.full(n_topics, 0.1), size=n_docs)
    ntok = r.poisson(mean_len, size=n_docs).astype(np.int32)
    offsets = np.zeros(n_docs + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(ntok)
    total = int(offsets[-1])
    doc = np.repeat(np.arange(n_docs), ntok)
    zt = (r.random(total)[:, None] > np.cumsum(theta, axis=1)[doc]).sum(axis=1)
    zt = np.minimum(zt, n_topics - 1)
    cphi = np.cumsum(phi, axis=1)
    words = np.empty(total, dtype=np.int32)
    u = r.random(total)
    for k in range(n_topics):
        sel = np.nonzero(zt == k)[0]
        words[sel] = np.minimum(np.searchsorted(cphi[k], u[sel], side="right"), n_vocab - 1)
    z0 = r.integers(0, n_topics, size=total).astype(np.int32)
    return dict(n_docs=n_docs, n_topics=n_topics, n_vocab=n_vocab, offsets=offsets,
                words=words, z0=z0, ntok=ntok)


def step_params(n: int, seed: int = WORKLOAD_SEED):
    """Per-chain parameters for one-at-a-time calls: U(a,b), N(mu,sigma),
    Exp(lambda), Gamma(alpha) with alpha log-uniform on [0.05, 5000]."""
    r = _rng(seed, 7)
    a = r.normal(0.0, 3.0, n).astype(np.float32)
    b = (a + r.exponential(2.0, n) + 1e-3).astype(np.float32)
    mu = r.normal(0.0, 5.0, n).astype(np.float32)
    sigma = r.exponential(1.0, n).astype(np.float32) + np.float32(1e-3)
    lam = np.exp(r.uniform(np.log(1e-3), np.log(1e3), n)).astype(np.float32)
    alpha = np.exp(r.uniform(np.log(0.05), np.log(5000.0), n)).astype(np.float32)
    return dict(a=a, b=b, mu=mu, sigma=sigma, lam=lam, alpha=alpha)


def dirichlet_items(n_items: int, kmin: int = 1, kmax: int = 300, seed: int = WORKLOAD_SEED):
    """Ragged Dirichlet items: K_i ~ U{kmin..kmax}, alpha log-uniform on
    [0.05, 50]."""
    r = _rng(seed, 8)
    K = r.integers(kmin, kmax + 1, size=n_items).astype(np.int32)
    offsets = np.zeros(n_items + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(K)
    alpha = np.exp(r.uniform(np.log(0.05), np.log(50.0), int(offsets[-1]))).astype(np.float32)
    return dict(offsets=offsets, alpha=alpha, K=K)


SERVED_KINDS = ("uniform", "normal", "exponential", "gamma", "dirichlet")


def _log_uniform_int(r: np.random.Generator, lo: int, hi: int, n: int) -> np.ndarray:
    """round(exp(U ln lo + (1 - U) ln hi)), clamped to [lo, hi]."""
    u = r.random(n)
    v = np.rint(np.exp(u * np.log(lo) + (1.0 - u) * np.log(hi)))
    return np.clip(v, lo, hi).astype(np.int64)


def served_requests(n_requests: int, chains_max: int = 65536, steps_max: int = 10000,
                    seed: int = WORKLOAD_SEED):
    """A mixed request stream for the served form: per request a kind drawn
    uniformly from SERVED_KINDS, chains log-uniform in [1, chains_max], steps
    log-uniform in [10, steps_max], and a stream seed.  Per kind the chain
    model: uniform -> the triangle chain (fp64), normal -> the s-chain with
    its exponential, exponential -> e' ~ Exp(1 + e^2), gamma -> gamma chains
    with alpha_0 log-uniform on [0.1, 100], dirichlet -> LDA documents (the
    chains are documents, the steps sweeps) with K ~ U{8..256} and
    n ~ Poisson(200) tokens.  Arrival times are not drawn here."""
    r = _rng(seed, 9)
    kind = r.integers(0, len(SERVED_KINDS), n_requests)
    chains = _log_uniform_int(r, 1, chains_max, n_requests)
    steps = _log_uniform_int(r, 10, steps_max, n_requests)
    seeds = r.integers(0, 2**63, n_requests, dtype=np.int64).astype(np.uint64)
    out = []
    for i in range(n_requests):
        q = dict(kind=SERVED_KINDS[kind[i]], chains=int(chains[i]), steps=int(steps[i]),
                 seed=int(seeds[i]))
        if q["kind"] == "gamma":
            q["alpha0"] = (0.1 * np.power(1000.0, r.random(q["chains"]))).astype(np.float32)
        elif q["kind"] == "dirichlet":
            K = r.integers(8, 257, q["chains"]).astype(np.int32)
            q["ntok"] = r.poisson(200.0, q["chains"]).astype(np.int32)
            q["offsets"] = np.zeros(q["chains"] + 1, dtype=np.int32)
            q["offsets"][1:] = np.cumsum(K)
        out.append(q)
    return out


def poisson_arrivals(n: int, rate_per_s: float, seed: int = WORKLOAD_SEED) -> np.ndarray:
    """Arrival offsets in seconds of a Poisson process at the given rate."""
    r = _rng(seed, 10)
    return np.cumsum(r.exponential(1.0 / rate_per_s, n))
