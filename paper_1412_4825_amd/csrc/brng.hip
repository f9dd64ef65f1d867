// brng: kernels and the C interface declared in include/brng.h.
//
// Kernels (gfx950, wave64, no matrix cores: nothing here is a contraction):
//   k_fill<K>        bulk refill of every unit's window (Sec. 1 batch call /
//                    Sec. 2.2 constructor fill): one Philox block per lane,
//                    one 128-bit store per block, coalesced per wave
//   k_step_*         one draw per chain per launch (the one-at-a-time call
//                    of Sec. 1 with the reducible transforms of Sec. 2.1)
//   k_gibbs<M>       all steps of every chain of one request
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/brng.h"
#include "lda_packed.hpp"

#ifndef LDA_WAVES_PER_EU
#define LDA_WAVES_PER_EU 5
#endif
#include "models.hpp"
#include "slots.hpp"

using namespace brng;

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_init_meta(Meta* meta, uint32_t n_units, uint64_t seed) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_units) return;
    Meta m;
    for (int k = 0; k < 4; ++k) {
        m.cur[k] = 0;
        m.wbase[k] = 0;
        m.wlen[k] = 0;
    }
    m.key_unit = i;
    m.pad = 0;
    m.key_seed = seed;
    meta[i] = m;
}

// Cursors from a device array [unit][4]; windows become empty.
__global__ void k_set_cursors(Meta* meta, uint32_t n_units, const uint64_t* cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_units) return;
    for (int k = 0; k < 4; ++k) {
        meta[i].cur[k] = cur[4 * (size_t)i + k];
        meta[i].wbase[k] = 0;
        meta[i].wlen[k] = 0;
    }
}

__global__ void k_get_cursors(const Meta* meta, uint32_t n_units, uint64_t* cur) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_units) return;
    for (int k = 0; k < 4; ++k) cur[4 * (size_t)i + k] = meta[i].cur[k];
}

constexpr int FILL_THREADS = 256;
constexpr int FILL_BPT = 4;  // blocks per thread

// Grid (x: window slices of FILL_THREADS * FILL_BPT blocks, y: unit).  The
// window starts at the unit's cursor rounded down to 64 blocks.
template <uint32_t KIND>
__global__ __launch_bounds__(FILL_THREADS) void k_fill(Meta* meta,
                                                       typename KindTraits<KIND>::T* pool,
                                                       uint32_t W) {
    constexpr int EPB = KindTraits<KIND>::EPB;
    const uint32_t unit = blockIdx.y;
    Meta* mp = meta + unit;
    const uint64_t cur = mp->cur[KIND];
    const uint64_t first = cur & ~(uint64_t)(64 * EPB - 1);
    const Key key = meta_key(*mp);
    const uint32_t nblk = W / EPB;
    uint4* dst = reinterpret_cast<uint4*>(pool + (size_t)unit * W);
    const uint64_t b0 = first / EPB;
    const uint32_t base = blockIdx.x * (FILL_THREADS * FILL_BPT) + threadIdx.x;
#pragma unroll
    for (int i = 0; i < FILL_BPT; ++i) {
        const uint32_t b = base + i * FILL_THREADS;
        if (b < nblk) dst[b] = gen_block<KIND>(key, b0 + b);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        mp->wbase[KIND] = first;
        mp->wlen[KIND] = W;
    }
}

// Raw words -> base deviates (the conversion half of the engine): thread i
// converts words [4i, 4i + 4).
template <uint32_t KIND>
__global__ __launch_bounds__(256) void k_convert(const uint4* words, uint64_t nblk, uint4* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nblk) out[i] = convert_block<KIND>(words[i]);
}

__device__ __forceinline__ uint32_t wave_in_block() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// One-at-a-time calls: one wave per unit of 64 chains.
template <uint32_t KIND, typename T>
__global__ __launch_bounds__(512) void k_step_uniform(Meta* meta, T* pool, uint32_t W,
                                                      uint32_t n, const T* a, const T* b,
                                                      T* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const T u = r.take(act);
    if (act) {
        const T lo = a[c];
        out[c] = lo + (b[c] - lo) * u;
    }
    r.close(meta[unit]);
}

__global__ __launch_bounds__(512) void k_step_normal(Meta* meta, float* pool, uint32_t W,
                                                     uint32_t n, const float* mu,
                                                     const float* sigma, float* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_N> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const float z = r.take(act);
    if (act) out[c] = fmaf(sigma[c], z, mu[c]);
    r.close(meta[unit]);
}

__global__ __launch_bounds__(512) void k_step_exp(Meta* meta, float* pool, uint32_t W, uint32_t n,
                                                  const float* lam, float* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_E> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const float e = r.take(act);
    if (act) out[c] = e / lam[c];
    r.close(meta[unit]);
}

// Laplace (GetLaplace, Sec. 2.2): mu + b (E1 - E2), two calls on the
// exponential pool.
__global__ __launch_bounds__(512) void k_step_laplace(Meta* meta, float* pool, uint32_t W,
                                                      uint32_t n, const float* mu, const float* b,
                                                      float* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_E> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const float e1 = r.take(act);
    const float e2 = r.take(act);
    if (act) {
        const float s = b[c];
        out[c] = mu[c] + (s * e1 - s * e2);
    }
    r.close(meta[unit]);
}

// Weibull (GetWeibull, Sec. 2.2): lambda E^(1/k) = lambda 2^(log2(E) / k),
// one call on the exponential pool.
__global__ __launch_bounds__(512) void k_step_weibull(Meta* meta, float* pool, uint32_t W,
                                                      uint32_t n, const float* lam, const float* k,
                                                      float* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_E> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const float e = r.take(act);
    if (act) out[c] = lam[c] * __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(e) / k[c]);
    r.close(meta[unit]);
}

// Poisson (a discrete getter: the expanded library of Sec. 3's future
// work), in double precision on the uniform pool.  lambda < 10: inversion
// with one uniform, k = min{k : u <= F(k)} with F accumulated from
// p_0 = exp(-lambda), p_k = p_{k-1} lambda / k.  lambda >= 10: Hormann's
// transformed rejection with squeeze (PTRS, 1993), two uniforms per attempt.
// Lanes take uniforms in rounds: one to every pending lane (lane order), then
// one more to every pending lane with lambda >= 10; a lane with lambda < 10
// is pending only in the first round.  lambda outside [0, 2^30] gives -1 and
// takes nothing.
struct Ptrs {
    double lam, loglam, a, b, invalpha, vr;
    __device__ __forceinline__ void setup(double l) {
        lam = l;
        loglam = log(l);
        b = 0.931 + 2.53 * sqrt(l);
        a = -0.059 + 0.02483 * b;
        invalpha = 1.1239 + 1.1328 / (b - 3.4);
        vr = 0.9277 - 3.6224 / (b - 2.0);
    }
    // one attempt with uniforms u, v: true and *k when accepted
    __device__ __forceinline__ bool attempt(double u, double v, int32_t* k) const {
        const double U = u - 0.5;
        const double us = 0.5 - fabs(U);
        const double kk = floor((2.0 * a / us + b) * U + lam + 0.43);
        if (us >= 0.07 && v <= vr) {
            *k = (int32_t)kk;
            return true;
        }
        if (kk < 0.0 || (us < 0.013 && v > us)) return false;
        const double lhs = log(v) + log(invalpha) - log(a / (us * us) + b);
        if (lhs <= -lam + kk * loglam - lgamma(kk + 1.0)) {
            *k = (int32_t)kk;
            return true;
        }
        return false;
    }
};

__device__ __forceinline__ int32_t poisson_invert(double lam, double u) {
    double p = exp(-lam), F = p;
    int32_t k = 0;
    while (u > F && k < 1000) {
        k += 1;
        p = p * lam / (double)k;
        F = F + p;
    }
    return k;
}

__global__ __launch_bounds__(512) void k_step_poisson(Meta* meta, float* pool, uint32_t W,
                                                      uint32_t n, const float* lam_in,
                                                      int32_t* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_U> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const double lam = act ? (double)lam_in[c] : -1.0;
    const bool valid = lam >= 0.0 && lam <= 0x1p30;  // false for NaN
    const bool large = valid && lam >= 10.0;
    Ptrs P;
    if (large) P.setup(lam);
    int32_t k = -1;
    bool pend = valid;
    for (uint32_t round = 0; round < (1u << 20); ++round) {
        if (wave_ballot(pend) == 0) break;
        const double u = (double)r.take(pend);
        const bool need_v = pend && large;
        const double v = (double)r.take(need_v);
        if (pend && !large) {
            k = poisson_invert(lam, u);
            pend = false;
        } else if (need_v) {
            int32_t kk;
            if (P.attempt(u, v, &kk)) {
                k = kk;
                pend = false;
            }
        }
    }
    if (act) out[c] = k;
    r.close(meta[unit]);
}

// Binomial (the second discrete getter), double precision on the uniform
// pool.  With p' = min(p, 1 - p) the draw is made for p' and mirrored
// (n - k) when p > 1/2.  n p' < 10: inversion with one uniform,
// k = min{k : u <= F(k)}, F accumulated from P_0 = exp(n ln(1 - p')),
// P_k = P_{k-1} (n - k + 1) / k * p'/(1 - p').  Otherwise Hormann's
// transformed rejection with decomposition (BTRD, 1993): an attempt's first
// uniform v accepts at once below u_r v_r; above, a second uniform is taken
// and the candidate k is accepted by the exact test ln(V alpha/(a/us^2 + b))
// <= ln P(k) - ln P(m), evaluated with ln Gamma.  Lanes take uniforms in
// rounds: one to every pending lane (lane order), then one more to every
// pending rejection-path lane whose first uniform was above u_r v_r; an
// inversion lane is pending only in the first round.  n < 0 or p outside
// [0, 1] gives -1 and takes nothing.
struct Btrd {
    double n, m, a, b, c, alpha, vr, urvr, logp, logq, lgn1, lpm;
    __device__ __forceinline__ double lp(double k) const {
        return lgn1 - lgamma(k + 1.0) - lgamma(n - k + 1.0) + k * logp + (n - k) * logq;
    }
    __device__ __forceinline__ void setup(int32_t ni, double p) {
        const double q = 1.0 - p;
        n = (double)ni;
        m = floor((n + 1.0) * p);
        const double spq = sqrt(n * p * q);
        b = 1.15 + 2.53 * spq;
        a = -0.0873 + 0.0248 * b + 0.01 * p;
        c = n * p + 0.5;
        alpha = (2.83 + 5.1 / b) * spq;
        vr = 0.92 - 4.2 / b;
        urvr = 0.86 * vr;
        logp = log(p);
        logq = log1p(-p);
        lgn1 = lgamma(n + 1.0);
        lpm = lp(m);
    }
    // first uniform: 1 accepted with *k, -1 rejected, 0 a second is needed
    __device__ __forceinline__ int first(double v, int32_t* k) const {
        if (v > urvr) return 0;
        const double U = v / vr - 0.43;
        const double kk = floor((2.0 * a / (0.5 - fabs(U)) + b) * U + c);
        if (kk >= 0.0 && kk <= n) {
            *k = (int32_t)kk;
            return 1;
        }
        return -1;
    }
    __device__ __forceinline__ bool second(double v, double w, int32_t* k) const {
        double U, V;
        if (v >= vr) {
            U = w - 0.5;
            V = v;
        } else {
            U = v / vr - 0.93;
            U = (U >= 0.0 ? 0.5 : -0.5) - U;
            V = w * vr;
        }
        const double us = 0.5 - fabs(U);
        const double x = (2.0 * a / us + b) * U + c;
        if (!(x >= 0.0 && x < n + 1.0)) return false;
        const double kk = floor(x);
        if (log(V * alpha / (a / (us * us) + b)) <= lp(kk) - lpm) {
            *k = (int32_t)kk;
            return true;
        }
        return false;
    }
};

__device__ __forceinline__ int32_t binomial_invert(int32_t n, double p, double u) {
    const double s = p / (1.0 - p);
    double P = exp((double)n * log1p(-p)), F = P;
    int32_t k = 0;
    while (u > F && k < n) {
        k += 1;
        P = P * (double)(n - k + 1) / (double)k * s;
        F = F + P;
    }
    return k;
}

// One binomial call over a wave: every lane with `act` draws
// Binomial(n, p) (-1 for n < 0 or p outside [0, 1]); the lanes take their
// uniforms in the rounds described above.  Called by every lane of the wave.
__device__ __forceinline__ int32_t binomial_call(DirectReader<KIND_U>& r, int32_t n, double p,
                                                 bool act) {
    const bool valid = act && n >= 0 && p >= 0.0 && p <= 1.0;  // false for NaN
    const bool flip = p > 0.5;
    const double pp = flip ? 1.0 - p : p;
    const bool inv = valid && (double)n * pp < 10.0;
    Btrd B;
    if (valid && !inv) B.setup(n, pp);
    int32_t k = -1;
    bool pend = valid;
    for (uint32_t round = 0; round < (1u << 20); ++round) {
        if (wave_ballot(pend) == 0) break;
        const double v = (double)r.take(pend);
        int32_t kk = 0;
        int st = 0;  // 1 done, -1 attempt rejected, 0 needs a second uniform
        if (pend) {
            if (inv) {
                kk = binomial_invert(n, pp, v);
                st = 1;
            } else {
                st = B.first(v, &kk);
            }
        }
        const bool need_w = pend && st == 0;
        const double w = (double)r.take(need_w);
        if (need_w) st = B.second(v, w, &kk) ? 1 : -1;
        if (pend && st == 1) {
            k = flip ? n - kk : kk;
            pend = false;
        }
    }
    return k;
}

__global__ __launch_bounds__(512) void k_step_binomial(Meta* meta, float* pool, uint32_t W,
                                                       uint32_t n_ch, const int32_t* n_in,
                                                       const float* p_in, int32_t* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n_ch) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n_ch;
    DirectReader<KIND_U> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    const int32_t k = binomial_call(r, act ? n_in[c] : -1, act ? (double)p_in[c] : 0.0, act);
    if (act) out[c] = k;
    r.close(meta[unit]);
}

// Multinomial by conditional binomials (the discrete library of Sec. 3's
// future work), one item per lane: x_k ~ Binomial(n - x_0 - ... - x_{k-1},
// p_k / S_k) for k < K - 1 and x_{K-1} the rest, where S_0 = p_0 + ... +
// p_{K-1} (index order, double precision) and S_{k+1} = S_k - p_k; S_k <= 0
// gives probability 0 and a quotient above 1 is taken as 1.  Component k of
// every item that draws one is one binomial call over the wave.  An item
// with n < 0, K < 1 or a weight that is negative or not finite gets -1 in
// every component and draws nothing.
__global__ __launch_bounds__(512) void k_step_multinomial(Meta* meta, float* pool, uint32_t W,
                                                          uint32_t n_items, const int32_t* offsets,
                                                          const int32_t* n_in, const float* w_in,
                                                          int32_t* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n_items) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n_items;
    DirectReader<KIND_U> r;
    r.open(meta[unit], pool + (size_t)unit * W, W);
    int32_t off = 0, K = 0, rem = -1;
    if (act) {
        off = offsets[c];
        K = offsets[c + 1] - off;
        rem = n_in[c];
    }
    bool ok = act && rem >= 0 && K >= 1;
    double S = 0.0;
    for (int32_t j = 0; ok && j < K; ++j) {
        const double wj = (double)w_in[off + j];
        ok = wj >= 0.0 && wj < INFINITY;
        S += wj;
    }
    const int32_t kmax = wave_minmax<true>(ok ? K : 0);
    for (int32_t k = 0; k + 1 < kmax; ++k) {
        const bool draw = ok && k + 1 < K;
        double q = 0.0;
        if (draw) {
            const double wk = (double)w_in[off + k];
            q = S > 0.0 ? wk / S : 0.0;
            q = q > 1.0 ? 1.0 : q;
            S -= wk;
        }
        const int32_t x = binomial_call(r, rem, q, draw);
        if (draw) {
            out[off + k] = x;
            rem -= x;
        }
    }
    if (ok)
        out[off + K - 1] = rem;
    else if (act)
        for (int32_t j = 0; j < K; ++j) out[off + j] = -1;
    r.close(meta[unit]);
}

__global__ __launch_bounds__(512) void k_step_gamma(Meta* meta, Pools P, uint32_t n,
                                                    const float* alpha, float* out) {
    const uint32_t unit = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (unit * 64 >= n) return;
    const uint32_t c = unit * 64 + lane_id();
    const bool act = c < n;
    DirectReader<KIND_N> rn;
    DirectReader<KIND_E> re;
    rn.open(meta[unit], P.n + (size_t)unit * P.W[KIND_N], P.W[KIND_N]);
    re.open(meta[unit], P.e + (size_t)unit * P.W[KIND_E], P.W[KIND_E]);
    OneEachSrc src;
    src.want = act ? 1 : 0;
    src.alpha = act ? alpha[c] : 1.0f;
    src.g = 0.0f;
    gamma_rounds<false>(rn, re, src, 4096u);
    if (act) out[c] = src.g;
    rn.close(meta[unit]);
    re.close(meta[unit]);
}

// Dirichlet: one wave per item, any K (the component gammas go to `out`,
// then are scaled by their sum, accumulated in the same order as in the LDA
// model).
// One Dirichlet draw by unit `unit` (one wave): shapes alpha[k], or base +
// cnt[k] when alpha is null, for K components; the normalised draw goes to
// out[k * os], k < K.  Gammas in rounds (gamma_rounds), straight from the
// windows.
__device__ void dirichlet_unit(Meta* meta, const Pools& P, uint32_t unit, int K,
                               const float* alpha, const int32_t* cnt, float base, float* out,
                               int os = 1) {
    const uint32_t lane = lane_id();
    DirectReader<KIND_N> rn;
    DirectReader<KIND_E> re;
    rn.open(meta[unit], P.n + (size_t)unit * P.W[KIND_N], P.W[KIND_N]);
    re.open(meta[unit], P.e + (size_t)unit * P.W[KIND_E], P.W[KIND_E]);
    CompSrc src;
    src.K = K;
    src.alpha = alpha;
    src.cnt = cnt;
    src.base = base;
    src.y = out;
    src.ys = os;
    gamma_rounds<false>(rn, re, src, 4096u + 64u * (uint32_t)min(K, 1 << 24));
    // component gammas were written by whichever lane drew them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    float part = 0.0f;
    for (int b0 = 0; b0 < K; b0 += 64) {
        const int k = b0 + (int)lane;
        if (k < K) part += out[(size_t)k * os];
    }
    const float S = wave_sum(part);
    for (int b0 = 0; b0 < K; b0 += 64) {
        const int k = b0 + (int)lane;
        if (k < K) out[(size_t)k * os] = S > 0.0f ? out[(size_t)k * os] / S : 0.0f;
    }
    rn.close(meta[unit]);
    re.close(meta[unit]);
}

__global__ __launch_bounds__(512) void k_step_dirichlet(Meta* meta, Pools P, uint32_t n_items,
                                                        const int32_t* offsets,
                                                        const float* alpha, float* out) {
    const uint32_t item = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (item >= n_items) return;
    const int32_t off = offsets[item];
    const int K = offsets[item + 1] - off;
    if (K < 1) return;
    dirichlet_unit(meta, P, item, K, alpha + off, nullptr, 0.0f, out + off);
}

// ---------------------------------------------------------------------------
// Full LDA: the uncollapsed Gibbs sampler of the LDA model whose Dirichlet
// redraws motivate the method (Sec. 1 and its footnote).  Per sweep,
// phi_k ~ Dir(beta + n_k.) for every topic, theta_d ~ Dir(alpha + n_d.) for
// every document, then every token's topic z ~ Cat(theta_d,k phi_k,w).
// Topic k's words [j LDAF_VBLOCK, (j + 1) LDAF_VBLOCK) are unit k nb + j
// (nb = ceil(V / LDAF_VBLOCK) blocks per topic), document d is unit K nb + d.
// Token indices are clamped to
// [0, n_tokens), so malformed offsets read nothing outside the arrays.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero_i32(int32_t* p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Counts of an assignment (n_dk and n_kw zero on entry); one wave per document.
__global__ __launch_bounds__(512) void k_ldaf_recount(uint32_t D, int K, int V,
                                                      const int32_t* doff, int32_t n_tokens,
                                                      const int32_t* words, const int32_t* z,
                                                      int32_t* ndk, int32_t* nkw) {
    const uint32_t d = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (d >= D) return;
    const int32_t a = max(doff[d], 0), b = min(doff[d + 1], n_tokens);
    for (int32_t i = a + (int32_t)lane_id(); i < b; i += 64) {
        const int32_t k = z[i], w = words[i];
        if (k >= 0 && k < K && w >= 0 && w < V) {
            atomicAdd(&ndk[(size_t)d * K + k], 1);
            atomicAdd(&nkw[(size_t)k * V + w], 1);
        }
    }
}

// The sweep's Dirichlets in one launch, one wave (and workgroup) each: the
// first K nb workgroups draw the topics' gammas, workgroup k nb + j those of
// topic k over words [j LDAF_VBLOCK, (j + 1) LDAF_VBLOCK) from unit k nb + j,
// the others theta_d ~ Dir(alpha + n_d.) (document d = block - K nb), so that
// the long topic draws run beside the many short document ones.  Every
// unit's pools are staged through LDS by the epoch readers of the LDA kernel
// (a topic block's thousands of components, or a document's up to 1,024,
// are many sequential rounds); phi is
// word-major ([V][K]), so that a token's K weights are one contiguous row.
// With one block per topic the wave also normalises phi_k; with more, each
// block leaves its gammas in phi and their fp32 sum in psum[k nb + j], and
// k_ldaf_phi_norm divides by the topic's total.
constexpr int LDAF_TOPIC_LDS = LdaRN::LDS_BYTES + LdaRE::LDS_BYTES;
constexpr int LDAF_VBLOCK = BRNG_LDAF_VBLOCK;
// The gammas of one unit's components (shapes base + cnt[c], c < n) into
// y[c ys], through the LDS epoch readers.
__device__ __forceinline__ void ldaf_gammas(Meta* meta, const Pools& P, uint32_t unit,
                                            unsigned char* lds, int n, const int32_t* cnt,
                                            float base, float* y, int ys) {
    Meta m = meta[unit];
    // the key words feed the scalar key schedule: make them provably uniform
    m.key_unit = __builtin_amdgcn_readfirstlane(m.key_unit);
    m.key_seed = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(m.key_seed >> 32)) << 32) |
                 (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)m.key_seed);
    LdaRN rn;
    LdaRE re;
    rn.open(m, P.n + (size_t)unit * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)unit * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + LdaRN::LDS_BYTES));
    CompSrc src;
    src.K = n;
    src.alpha = nullptr;
    src.cnt = cnt;
    src.base = base;
    src.y = y;
    src.ys = ys;
    gamma_rounds<true, LDA_EPOCH>(rn, re, src, 4096u + 64u * (uint32_t)n);
    rn.close(meta[unit]);
    re.close(meta[unit]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

__global__ __launch_bounds__(64) void k_ldaf_dirichlets(Meta* meta, Pools P, uint32_t D, int K,
                                                        int V, uint32_t nb, float alpha,
                                                        float beta, const int32_t* ndk,
                                                        const int32_t* nkw, float* theta,
                                                        float* phi, float* psum) {
    __shared__ __align__(16) unsigned char lds[LDAF_TOPIC_LDS];
    const uint32_t blk = blockIdx.x;
    const uint32_t n_topic_units = (uint32_t)K * nb;
    const uint32_t lane = lane_id();
    if (blk >= n_topic_units) {
        // theta_d ~ Dir(alpha + n_d.), normalised by the sum of its gammas
        const uint32_t d = blk - n_topic_units;
        if (d >= D) return;
        float* out = theta + (size_t)d * K;
        ldaf_gammas(meta, P, blk, lds, K, ndk + (size_t)d * K, alpha, out, 1);
        float part = 0.0f;
        for (int b0 = 0; b0 < K; b0 += 64) {
            const int k = b0 + (int)lane;
            if (k < K) part += out[k];
        }
        const float S = wave_sum(part);
        for (int b0 = 0; b0 < K; b0 += 64) {
            const int k = b0 + (int)lane;
            if (k < K) out[k] = S > 0.0f ? out[k] / S : 0.0f;
        }
        return;
    }
    const uint32_t k = blk / nb, j = blk - k * nb;
    const int c0 = (int)j * LDAF_VBLOCK;
    const int Vb = min(LDAF_VBLOCK, V - c0);
    float* out = phi + (size_t)c0 * K + k;
    ldaf_gammas(meta, P, blk, lds, Vb, nkw + (size_t)k * V + c0, beta, out, K);
    float part = 0.0f;
    for (int b0 = 0; b0 < Vb; b0 += 64) {
        const int c = b0 + (int)lane;
        if (c < Vb) part += out[(size_t)c * K];
    }
    const float S = wave_sum(part);
    if (nb == 1) {
        for (int b0 = 0; b0 < Vb; b0 += 64) {
            const int c = b0 + (int)lane;
            if (c < Vb) out[(size_t)c * K] = S > 0.0f ? out[(size_t)c * K] / S : 0.0f;
        }
    } else if (lane == 0) {
        psum[blk] = S;
    }
}

// phi[w][k] /= sum over topic k's blocks of psum (in block order, fp32):
// every workgroup first forms the K totals in LDS, then divides a
// grid-strided share of the [V][K] array.
__global__ __launch_bounds__(256) void k_ldaf_phi_norm(int K, int V, uint32_t nb,
                                                       const float* psum, float* phi) {
    __shared__ float tot[BRNG_LDAF_KMAX];
    const uint32_t t = threadIdx.x;
    for (uint32_t k = t; k < (uint32_t)K; k += blockDim.x) {
        float S = 0.0f;
        for (uint32_t j = 0; j < nb; ++j) S += psum[k * nb + j];
        tot[k] = S;
    }
    __syncthreads();
    const uint32_t n = (uint32_t)V * (uint32_t)K;  // below 2^32 (checked by the caller)
    for (uint32_t i = blockIdx.x * blockDim.x + t; i < n; i += gridDim.x * blockDim.x) {
        const float S = tot[i % (uint32_t)K];
        phi[i] = S > 0.0f ? phi[i] / S : 0.0f;
    }
}

// One uniform per token of document d (token order; theta_d drawn by the
// Dirichlet launch before) and the token's topic: p_k = theta_k phi_w,k in
// fp32, q_k = rint(p_k 2^(24 - e)) with max p = f 2^e, f in [1/2, 1) (an
// exact scaling; all 1 when max p is not positive), C_k = q_0 + ... + q_k,
// j = (u 2^24 - 1) / 2, t = (j C_{K-1}) >> 23, z = the number of k with
// C_k <= t.  A word outside [0, V) gets z = -1 and no count but still takes
// its uniform.  The uniforms are taken 64 at a time (one per lane, in token
// order), and lane l then works out the topic of token i0 + l by itself,
// walking the K topics: its phi row (16-byte loads where rows are aligned),
// theta from LDS (one broadcast read per four topics), the largest p as
// int32 bits (the order a lane-parallel maximum over the topics, zeros of
// absent topics included, would give the same), the q_k and their integer
// sums.  A maximum and integer sums do not depend on their order, so the
// topic is the same, bit for bit, as from any other arrangement of the rule.
// KP: K padded to 16, 32 or 64 (the lane's registers are indexed
// statically; padded topics weigh 0 and are never counted); FULL: K = KP (no
// padded topics, no selects).  A token's row is read with all its loads in
// flight together.  New n_d. in place (LDS counts), n_kw added atomically
// (zero on entry), once per token.
template <int KP, bool FULL>
__global__ __launch_bounds__(512) void k_ldaf_docs(Meta* meta, Pools P, uint32_t D, int K, int V,
                                                   uint32_t nb, const int32_t* doff,
                                                   int32_t n_tokens,
                                                   const int32_t* words, const float* phi,
                                                   const float* theta, int32_t* z, int32_t* ndk,
                                                   int32_t* nkw) {
    static_assert(KP == 16 || KP == 32 || KP == 64, "topics padded to 16, 32 or 64");
    extern __shared__ int32_t ldaf_cnt[];
    const uint32_t d = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (d >= D) return;
    const uint32_t lane = lane_id();
    const uint32_t unit = (uint32_t)K * nb + d;
    int32_t* cnt = ldaf_cnt + 128 * wave_in_block();  // tokens per topic
    float* thl = reinterpret_cast<float*>(cnt + 64);  // theta_d, zero past K
    const float* th_row = theta + (size_t)d * K;
    int32_t* ndk_row = ndk + (size_t)d * K;
    cnt[lane] = 0;
    thl[lane] = (int)lane < K ? th_row[lane] : 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // rows start 16-byte aligned (and hold whole groups of four)
    const bool v4 = (K & 3) == 0 && ((uintptr_t)phi & 15u) == 0;
    const int32_t mb0 = K < 64 ? 0 : INT32_MIN;  // absent topics' zeros
    DirectReader<KIND_U> ru;
    ru.open(meta[unit], P.u + (size_t)unit * P.W[KIND_U], P.W[KIND_U]);
    const int32_t a = max(doff[d], 0), b = min(doff[d + 1], n_tokens);
    for (int32_t i0 = a; i0 < b; i0 += 64) {
        const int32_t i = i0 + (int32_t)lane;
        const bool act = i < b;
        const int32_t wl = act ? words[i] : -1;  // in flight during the take
        const float u = ru.take(act);
        const uint32_t j = (((uint32_t)(u * 16777216.0f)) - 1u) >> 1;
        const bool ok = wl >= 0 && wl < V;
        const float* row = phi + (size_t)(ok ? wl : 0) * K;  // row 0 stands in
        // K through an empty asm: the padding tests below are made where they
        // are used instead of being kept, one per topic, across the loop
        int Kx = __builtin_amdgcn_readfirstlane(K);
        asm volatile("" : "+s"(Kx));
        // the row: every load issued before any is used (padded topics read
        // a topic of the row and are zeroed below)
        float ph[KP];
        if (v4) {
#pragma unroll
            for (int k = 0; k < KP; k += 4) {
                const int kc = FULL ? k : min(k, Kx - 4);
                const float4 r4 = *reinterpret_cast<const float4*>(row + kc);
                ph[k] = r4.x;
                ph[k + 1] = r4.y;
                ph[k + 2] = r4.z;
                ph[k + 3] = r4.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < KP; ++k) ph[k] = row[FULL ? k : min(k, Kx - 1)];
        }
        float p[KP];
        int32_t mb = mb0;
#pragma unroll
        for (int k = 0; k < KP; k += 4) {
            const float4 t4 = *reinterpret_cast<const float4*>(thl + k);
            const float tk[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = tk[e] * ph[k + e];
                if (!FULL) v = k + e < Kx ? v : 0.0f;
                p[k + e] = v;
                mb = max(mb, __float_as_int(v));
            }
        }
        // largest p positive: q_k = rint(p_k 2^(24 - e)) (absent topics 0,
        // and Q >= 2^23 > t, so they are never counted); otherwise every
        // topic weighs 1, C_k = k + 1, Q = K and z = t
        const float m = __int_as_float(mb);
        const bool pos = m > 0.0f;
        const int sh = 24 - __builtin_amdgcn_frexp_expf(m);
        uint32_t q[KP];
        uint32_t Q = 0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            q[k] = (uint32_t)rintf(ldexpf(p[k], sh));
            Q += q[k];
        }
        const uint32_t t = (uint32_t)(((uint64_t)j * (pos ? Q : (uint32_t)K)) >> 23);
        uint32_t C = 0;
        int32_t zt = 0;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            C += q[k];
            zt += C <= t ? 1 : 0;
        }
        if (!pos) zt = (int32_t)t;
        const int32_t zl = ok ? zt : -1;
        if (act) z[i] = zl;
        if (zl >= 0) {
            atomicAdd(&cnt[zl], 1);
            atomicAdd(&nkw[(size_t)zl * V + wl], 1);
        }
    }
    ru.close(meta[unit]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if ((int)lane < K) ndk_row[lane] = cnt[lane];
}

// Documents of more than 64 topics (up to BRNG_LDAF_KMAX): the same rule and
// the same order of uniforms as k_ldaf_docs, one token per lane, but a lane's
// K weights do not fit its registers, so it forms them three times from its
// phi row (for the largest, the total and the count), 32 topics at a time
// with their row loads in flight together; the count stops once no lane's
// prefix sum is still <= its t (the sums only grow).  LDS per wave: the
// counts and theta_d, K rounded up to 4 each.
__global__ __launch_bounds__(512) void k_ldaf_docs_wide(Meta* meta, Pools P, uint32_t D, int K,
                                                        int V, uint32_t nb, const int32_t* doff,
                                                        int32_t n_tokens, const int32_t* words,
                                                        const float* phi, const float* theta,
                                                        int32_t* z, int32_t* ndk, int32_t* nkw) {
    extern __shared__ int32_t ldaf_cnt[];
    const uint32_t d = blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (d >= D) return;
    const uint32_t lane = lane_id();
    const uint32_t unit = (uint32_t)K * nb + d;
    const int K4 = (K + 3) & ~3;
    int32_t* cnt = ldaf_cnt + 2 * K4 * (int)wave_in_block();  // tokens per topic
    float* thl = reinterpret_cast<float*>(cnt + K4);           // theta_d, zero past K
    const float* th_row = theta + (size_t)d * K;
    int32_t* ndk_row = ndk + (size_t)d * K;
    for (int k = (int)lane; k < K4; k += 64) {
        cnt[k] = 0;
        thl[k] = k < K ? th_row[k] : 0.0f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool v4 = (K & 3) == 0 && ((uintptr_t)phi & 15u) == 0;
    const int K32 = K & ~31;  // topics in whole groups of 32
    const int Kf = K & ~3;    // and of four
    DirectReader<KIND_U> ru;
    ru.open(meta[unit], P.u + (size_t)unit * P.W[KIND_U], P.W[KIND_U]);
    const int32_t a = max(doff[d], 0), b = min(doff[d + 1], n_tokens);
    for (int32_t i0 = a; i0 < b; i0 += 64) {
        const int32_t i = i0 + (int32_t)lane;
        const bool act = i < b;
        const int32_t wl = act ? words[i] : -1;  // in flight during the take
        const float u = ru.take(act);
        const uint32_t j = (((uint32_t)(u * 16777216.0f)) - 1u) >> 1;
        const bool ok = wl >= 0 && wl < V;
        const float* row = phi + (size_t)(ok ? wl : 0) * K;  // row 0 stands in
        // weights of topics k .. k + G - 1 (k + G <= K), the row's loads
        // issued together
        auto group = [&](int k, auto gc, float* p) {
            constexpr int G = decltype(gc)::value;
            float ph[G];
            if (v4) {
#pragma unroll
                for (int g = 0; g < G; g += 4) {
                    const float4 r4 = *reinterpret_cast<const float4*>(row + k + g);
                    ph[g] = r4.x;
                    ph[g + 1] = r4.y;
                    ph[g + 2] = r4.z;
                    ph[g + 3] = r4.w;
                }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) ph[g] = row[k + g];
            }
#pragma unroll
            for (int g = 0; g < G; g += 4) {
                const float4 t4 = *reinterpret_cast<const float4*>(thl + k + g);
                p[g] = t4.x * ph[g];
                p[g + 1] = t4.y * ph[g + 1];
                p[g + 2] = t4.z * ph[g + 2];
                p[g + 3] = t4.w * ph[g + 3];
            }
        };
        using G32 = std::integral_constant<int, 32>;
        using G4 = std::integral_constant<int, 4>;
        // the weight of topic k (k < K), one at a time (the last partial group)
        auto one = [&](int k) { return thl[k] * row[k]; };
        // topics [0, K32) in groups of 32, [K32, Kf) in groups of 4, then singly
        int32_t mb = INT32_MIN;
        {
            int k = 0;
            for (; k < K32; k += 32) {
                float p[32];
                group(k, G32{}, p);
#pragma unroll
                for (int e = 0; e < 32; ++e) mb = max(mb, __float_as_int(p[e]));
            }
            for (; k < Kf; k += 4) {
                float p[4];
                group(k, G4{}, p);
#pragma unroll
                for (int e = 0; e < 4; ++e) mb = max(mb, __float_as_int(p[e]));
            }
            for (; k < K; ++k) mb = max(mb, __float_as_int(one(k)));
        }
        const float m = __int_as_float(mb);
        const bool pos = m > 0.0f;
        const int sh = 24 - __builtin_amdgcn_frexp_expf(m);
        auto qof = [&](float p) { return (uint32_t)rintf(ldexpf(p, sh)); };
        uint32_t Q = 0;
        {
            int k = 0;
            for (; k < K32; k += 32) {
                float p[32];
                group(k, G32{}, p);
#pragma unroll
                for (int e = 0; e < 32; ++e) Q += qof(p[e]);
            }
            for (; k < Kf; k += 4) {
                float p[4];
                group(k, G4{}, p);
#pragma unroll
                for (int e = 0; e < 4; ++e) Q += qof(p[e]);
            }
            for (; k < K; ++k) Q += qof(one(k));
        }
        // every topic weighs 1 when the largest weight is not positive:
        // C_k = k + 1, Q = K, z = t
        const uint32_t t = (uint32_t)(((uint64_t)j * (pos ? Q : (uint32_t)K)) >> 23);
        int32_t zt = (int32_t)t;
        if (wave_ballot(ok && pos) != 0) {
            uint32_t C = 0;
            int32_t cz = 0;
            bool more = true;  // some lane's prefix sum is still <= its t
            int k = 0;
            for (; more && k < K32; k += 32) {
                float p[32];
                group(k, G32{}, p);
#pragma unroll
                for (int e = 0; e < 32; ++e) {
                    C += qof(p[e]);
                    cz += C <= t ? 1 : 0;
                }
                more = wave_ballot(ok && pos && C <= t) != 0;
            }
            for (; more && k < Kf; k += 4) {
                float p[4];
                group(k, G4{}, p);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    C += qof(p[e]);
                    cz += C <= t ? 1 : 0;
                }
                more = wave_ballot(ok && pos && C <= t) != 0;
            }
            for (; more && k < K; ++k) {
                C += qof(one(k));
                cz += C <= t ? 1 : 0;
            }
            if (pos) zt = cz;
        }
        const int32_t zl = ok ? zt : -1;
        if (act) z[i] = zl;
        if (zl >= 0) {
            atomicAdd(&cnt[zl], 1);
            atomicAdd(&nkw[(size_t)zl * V + wl], 1);
        }
    }
    ru.close(meta[unit]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int k = (int)lane; k < K; k += 64) ndk_row[k] = cnt[k];
}

template <int MODEL>
__device__ __forceinline__ void run_unit(const DescDev& D, Meta* meta, const Pools& P,
                                         uint32_t local, unsigned char* lds) {
    Meta* mp = meta + D.unit_base + local;
    if constexpr (MODEL == M_TRIANGLE) unit_triangle(D, mp, P, local, lds);
    if constexpr (MODEL == M_NORMEXP) unit_normexp(D, mp, P, local, lds);
    if constexpr (MODEL == M_GAMMA) {
        if (D.sums)  // the sums path, kept out of the rounds of runs without
            unit_gamma<true>(D, mp, P, local, lds);
        else
            unit_gamma<false>(D, mp, P, local, lds);
    }
    if constexpr (MODEL == M_LDA) unit_lda(D, mp, P, local, lds);
    if constexpr (MODEL == M_EXPCHAIN) unit_expchain(D, mp, P, local, lds);
}

__host__ __device__ constexpr int model_lds_bytes(int model) {
    return model == M_LDA        ? LDA_LDS_BYTES
           : model == M_NORMEXP  ? NORMEXP_LDS_BYTES
           : model == M_EXPCHAIN ? EXPCHAIN_LDS_BYTES
           : model == M_GAMMA    ? GAMMA_LDS_BYTES
                                 : RING_BYTES;
}

// Documents the LDA kernels cannot serve: K outside [1, 256], negative
// token counts, or traces too narrow for their components.  Such a document
// gets -1 in every count of its state (when it has components) and nothing
// else changes.
__device__ __forceinline__ bool lda_doc_ok(const DescDev& D, uint32_t doc) {
    const int32_t off = D.offsets[doc];
    const int K = D.offsets[doc + 1] - off;
    const bool fits = (!D.trace && !D.trace2) || (off >= 0 && (int64_t)off + K <= D.stride);
    return K >= 1 && K <= LDA_KMAX && D.ntok[doc] >= 0 && fits;
}

// Mark an unserved document (threads t of n write its counts).
__device__ __forceinline__ void lda_doc_reject(const DescDev& D, uint32_t doc, uint32_t t,
                                               uint32_t n) {
    const int32_t off = D.offsets[doc];
    const int K = D.offsets[doc + 1] - off;
    if (off < 0 || K < 1) return;
    int32_t* counts = reinterpret_cast<int32_t*>(D.state) + off;
    for (int k = (int)t; k < K; k += (int)n) counts[k] = -1;
}

// The plain LDA launch runs from a plan that a one-workgroup kernel builds
// first: the request's documents in six lists by component count, each in
// index order, laid out so that the most work per wave starts first: up to
// 8 components (eight documents to a wave), 129..256, 9..16 (four to a
// wave), 65..128, 33..64 and 17..32 (one to a wave).  plan[0..5] = the
// lists' lengths, list j at plan + PLAN_HEAD + j n_docs.  Documents that
// cannot be served are marked here.  (The order changes no result: every
// document is its own unit.)
constexpr int PLAN_HEAD = 8;
constexpr int PLAN_LISTS = 6;
constexpr int PLAN_THREADS = 1024;

__device__ __forceinline__ int plan_list(int K) {
    return K <= 8 ? 0 : K <= 16 ? 2 : K <= 32 ? 5 : K <= 64 ? 4 : K <= 128 ? 3 : 1;
}

__global__ __launch_bounds__(PLAN_THREADS) void k_lda_plan(DescDev D, int32_t* plan) {
    __shared__ uint32_t wc[PLAN_THREADS / 64][PLAN_LISTS];
    __shared__ uint32_t base[PLAN_LISTS];
    constexpr int AHEAD = 8;  // blocks of documents whose inputs are loaded together
    const uint32_t n = D.n_units, tid = threadIdx.x, wv = tid / 64;
    if (tid < PLAN_LISTS) base[tid] = 0;
    __syncthreads();
    int32_t* lists = plan + PLAN_HEAD;
    for (uint32_t c0 = 0; c0 < n; c0 += AHEAD * PLAN_THREADS) {
        int32_t o0[AHEAD], o1[AHEAD], nt[AHEAD];
#pragma unroll
        for (int i = 0; i < AHEAD; ++i) {
            const uint32_t doc = c0 + (uint32_t)i * PLAN_THREADS + tid;
            o0[i] = o1[i] = nt[i] = 0;
            if (doc < n) {
                o0[i] = D.offsets[doc];
                o1[i] = D.offsets[doc + 1];
                nt[i] = D.ntok[doc];
            }
        }
#pragma unroll
        for (int i = 0; i < AHEAD; ++i) {
            const uint32_t b0 = c0 + (uint32_t)i * PLAN_THREADS;
            if (b0 >= n) break;
            const uint32_t doc = b0 + tid;
            int l = -1;
            if (doc < n) {
                const int K = o1[i] - o0[i];
                const bool fits = (!D.trace && !D.trace2) ||
                                  (o0[i] >= 0 && (int64_t)o0[i] + K <= D.stride);
                if (K >= 1 && K <= LDA_KMAX && nt[i] >= 0 && fits)
                    l = plan_list(K);
                else
                    lda_doc_reject(D, doc, 0, 1);
            }
            uint32_t rank = 0;
            for (int j = 0; j < PLAN_LISTS; ++j) {
                const uint64_t mk = __builtin_amdgcn_ballot_w64(l == j);
                if (l == j) rank = mask_rank(mk);
                if (lane_id() == 0) wc[wv][j] = (uint32_t)__popcll(mk);
            }
            __syncthreads();
            if (l >= 0) {
                uint32_t pos = base[l] + rank;
                for (uint32_t w = 0; w < wv; ++w) pos += wc[w][l];
                lists[(size_t)l * n + pos] = (int32_t)doc;
            }
            __syncthreads();
            if (tid < PLAN_LISTS) {
                uint32_t t = 0;
                for (uint32_t w = 0; w < PLAN_THREADS / 64; ++w) t += wc[w][tid];
                base[tid] += t;
            }
            __syncthreads();
        }
    }
    if (tid < PLAN_LISTS) plan[tid] = (int32_t)base[tid];
}

// Plain form: one launch per request, one wave per unit (LDA: waves as the
// plan lays them out: groups of small documents first, then one document
// per wave).
template <int MODEL>
__device__ __forceinline__ void gibbs_body(const DescDev& D, Meta* meta, const Pools& P,
                                           const int32_t* plan) {
    extern __shared__ __align__(16) unsigned char lds_all[];
    const uint32_t w = wave_in_block();
    const uint32_t local = blockIdx.x * (blockDim.x >> 6) + w;
    if (local >= D.n_units) return;
    unsigned char* lds = lds_all + w * model_lds_bytes(MODEL);
    if constexpr (MODEL == M_LDA) {
        // the lists in wave order, with documents per wave 8, 1, 4, 1, 1, 1
        const uint32_t n = D.n_units;
        uint32_t w = local;
        for (int j = 0; j < PLAN_LISTS; ++j) {
            const uint32_t len = (uint32_t)plan[j];
            const uint32_t per = j == 0 ? 8u : j == 2 ? 4u : 1u;
            const uint32_t waves = (len + per - 1) / per;
            if (w < waves) {
                const int32_t* list = plan + PLAN_HEAD + (size_t)j * n + per * w;
                const uint32_t cnt = min(per, len - per * w);
                if (j == 0)
                    unit_lda_packed<8>(D, meta, P, list, cnt, lds);
                else if (j == 2)
                    unit_lda_packed<16>(D, meta, P, list, cnt, lds);
                else
                    run_unit<M_LDA>(D, meta, P, (uint32_t)list[0], lds);
                return;
            }
            w -= waves;
        }
    } else {
        run_unit<MODEL>(D, meta, P, local, lds);
    }
}

template <int MODEL>
__global__ __launch_bounds__(512) void k_gibbs(DescDev D, Meta* meta, Pools P,
                                               const int32_t* plan) {
    gibbs_body<MODEL>(D, meta, P, plan);
}

// The LDA kernel is held to five waves per SIMD (at most 102 registers):
// its LDS allows that many, and its rounds gain from the extra latency
// hiding more than they lose to the tighter register budget.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(LDA_WAVES_PER_EU)))
void k_gibbs_lda(DescDev D, Meta* meta, Pools P, const int32_t* plan) {
    gibbs_body<M_LDA>(D, meta, P, plan);
}

// Batched and served form: the units of several requests in one launch.  A
// wave finds its request by binary search over the slots' unit prefix in the
// device table (the index is wave-uniform, so the search and the slot's
// fields are scalar loads).  MODEL is one model, or M_MIXED: the wave then
// runs its request's model.  lds_wave: LDS bytes per wave.
constexpr int M_MIXED = -1;

__device__ __forceinline__ int slot_lookup(const SlotDev* __restrict__ tab, uint32_t n,
                                           uint32_t g, uint32_t* first) {
    uint32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tab[mid].unit_end > g)
            hi = mid;
        else
            lo = mid + 1;
    }
    *first = lo ? tab[lo - 1].unit_end : 0u;
    return (int)lo;
}

// LDA documents run in index order here (the descriptor's document order
// is only a scheduling hint, used by the plain launch).
template <int MODEL>
__device__ __forceinline__ void run_slot_unit(const DescDev& D, Meta* meta, const Pools& P,
                                              uint32_t local, unsigned char* lds) {
    if (MODEL == M_LDA && !lda_doc_ok(D, local)) {
        lda_doc_reject(D, local, lane_id(), 64);
        return;
    }
    run_unit<MODEL>(D, meta, P, local, lds);
}

// A slot read through the constant address space, field by field: the table
// is read-only while a kernel runs (the copy launches before it wrote it), so
// the reads are uniform scalar loads and the fields land in scalar registers,
// as kernel arguments would.
typedef const SlotDev __attribute__((address_space(4))) ConstSlot;
static_assert(sizeof(DescDev) == 128 && sizeof(Pools) == 48,
              "load_slot copies every field of the descriptor and the pools");

__device__ __forceinline__ void load_slot(ConstSlot* p, DescDev& D, Pools& P, Meta*& meta) {
    D.model = p->D.model;
    D.n_chains = p->D.n_chains;
    D.unit_base = p->D.unit_base;
    D.flags = p->D.flags;
    D.seed = p->D.seed;
    D.max_steps = p->D.max_steps;
    D.n_units = p->D.n_units;
    D.steps = p->D.steps;
    D.perm = p->D.perm;
    D.state = p->D.state;
    D.trace = p->D.trace;
    D.trace2 = p->D.trace2;
    D.stride = p->D.stride;
    D.offsets = p->D.offsets;
    D.ntok = p->D.ntok;
    D.step0 = p->D.step0;
    D.max_rounds = p->D.max_rounds;
    D.progress = p->D.progress;
    D.unit_done = p->D.unit_done;
    D.sums = p->D.sums;
    P.u = p->P.u;
    P.n = p->P.n;
    P.e = p->P.e;
    P.u64 = p->P.u64;
#pragma unroll
    for (int k = 0; k < 4; ++k) P.W[k] = p->P.W[k];
    meta = p->meta;
}

template <int MODEL>
__device__ __forceinline__ void multi_body(const SlotDev* __restrict__ tab, uint32_t n,
                                           uint32_t total_units, uint32_t lds_wave) {
    extern __shared__ __align__(16) unsigned char lds_all[];
    const uint32_t w = wave_in_block();
    const uint32_t g = blockIdx.x * (blockDim.x >> 6) + w;
    if (g >= total_units) return;
    uint32_t first;
    const int i = slot_lookup(tab, n, g, &first);
    DescDev D;
    Pools P;
    Meta* meta;
    load_slot((ConstSlot*)(tab + i), D, P, meta);
    const uint32_t local = g - first;
    unsigned char* lds = lds_all + w * lds_wave;
    if constexpr (MODEL == M_MIXED) {
        switch (D.model) {
            case M_TRIANGLE: run_slot_unit<M_TRIANGLE>(D, meta, P, local, lds); break;
            case M_NORMEXP: run_slot_unit<M_NORMEXP>(D, meta, P, local, lds); break;
            case M_GAMMA: run_slot_unit<M_GAMMA>(D, meta, P, local, lds); break;
            case M_LDA: run_slot_unit<M_LDA>(D, meta, P, local, lds); break;
            case M_EXPCHAIN: run_slot_unit<M_EXPCHAIN>(D, meta, P, local, lds); break;
            default: break;
        }
    } else {
        run_slot_unit<MODEL>(D, meta, P, local, lds);
    }
}

template <int MODEL>
__global__ __launch_bounds__(512) void k_multi(const SlotDev* __restrict__ tab, uint32_t n,
                                               uint32_t total_units, uint32_t lds_wave) {
    multi_body<MODEL>(tab, n, total_units, lds_wave);
}

// The mixed kernel holds every model's code, so its register count is that
// of the largest (the normal/exponential pipeline); it is capped so that
// three waves fit per SIMD, as the gamma and LDA kernels' LDS allows.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
void k_mixed(const SlotDev* __restrict__ tab, uint32_t n, uint32_t total_units,
             uint32_t lds_wave) {
    multi_body<M_MIXED>(tab, n, total_units, lds_wave);
}

// Copy one chunk of slots into the device table (32-bit words).
__global__ __launch_bounds__(256) void k_put_slots(SlotDev* tab, const SlotChunk c) {
    const uint32_t words = c.n * (uint32_t)(sizeof(SlotDev) / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(c.s);
    uint32_t* dst = reinterpret_cast<uint32_t*>(tab + c.base);
    for (uint32_t k = threadIdx.x; k < words; k += blockDim.x) dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct brng_ctx {
    brng_config cfg;
    hipStream_t stream;
    uint32_t n_units;
    void* pool[4];
    Meta* meta;
    SlotDev* table;  // slots of the batched form (BRNG_BATCH_MAX entries)
    int32_t* lda_plan;  // plain LDA launches: PLAN_HEAD + PLAN_LISTS n_units int32
                        // (full LDA: the topic blocks' gamma sums)
    int wpb;
    int n_cu;
    // events for the next plain chain launch (brng_time_next_launch)
    hipEvent_t t_start = nullptr, t_stop = nullptr;
};

static thread_local int32_t g_last_hip = 0;

static brng_status hip_fail(hipError_t e) {
    g_last_hip = (int32_t)e;
    return BRNG_E_HIP;
}

#define HIPCHK(x)                                     \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return hip_fail(e_);    \
    } while (0)

static size_t kind_elem(int k) { return k == BRNG_U64 ? sizeof(double) : sizeof(float); }

static bool window_ok(uint32_t W) {
    return W == 0 || (W % BRNG_WINDOW_ALIGN == 0 && W >= BRNG_WINDOW_MIN);
}

static Pools make_pools(const brng_ctx* c) {
    Pools p;
    p.u = (float*)c->pool[BRNG_U];
    p.n = (float*)c->pool[BRNG_N];
    p.e = (float*)c->pool[BRNG_E];
    p.u64 = (double*)c->pool[BRNG_U64];
    for (int k = 0; k < 4; ++k) p.W[k] = c->cfg.window[k];
    return p;
}

static brng_status launch_fill(brng_ctx* c, int kind) {
    const uint32_t W = c->cfg.window[kind];
    const uint32_t epb = kind == BRNG_U64 ? 2 : 4;
    const uint32_t nblk = W / epb;
    dim3 grid((nblk + FILL_THREADS * FILL_BPT - 1) / (FILL_THREADS * FILL_BPT), c->n_units);
    switch (kind) {
        case BRNG_U:
            hipLaunchKernelGGL(k_fill<KIND_U>, grid, dim3(FILL_THREADS), 0, c->stream, c->meta,
                               (float*)c->pool[kind], W);
            break;
        case BRNG_N:
            hipLaunchKernelGGL(k_fill<KIND_N>, grid, dim3(FILL_THREADS), 0, c->stream, c->meta,
                               (float*)c->pool[kind], W);
            break;
        case BRNG_E:
            hipLaunchKernelGGL(k_fill<KIND_E>, grid, dim3(FILL_THREADS), 0, c->stream, c->meta,
                               (float*)c->pool[kind], W);
            break;
        default:
            hipLaunchKernelGGL(k_fill<KIND_U64>, grid, dim3(FILL_THREADS), 0, c->stream, c->meta,
                               (double*)c->pool[kind], W);
            break;
    }
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

static void free_ctx(brng_ctx* c) {
    if (!c) return;
    for (int k = 0; k < 4; ++k)
        if (c->pool[k]) (void)hipFree(c->pool[k]);
    if (c->meta) (void)hipFree(c->meta);
    if (c->table) (void)hipFree(c->table);
    if (c->lda_plan) (void)hipFree(c->lda_plan);
    delete c;
}

namespace brng {

int model_lds_bytes_host(int model) { return model_lds_bytes(model); }

uint32_t desc_unit_count(const brng_gibbs_desc& d) {
    return d.model == BRNG_MODEL_LDA ? d.n_chains : (d.n_chains + 63) / 64;
}

DescDev desc_to_device(const brng_gibbs_desc& d) {
    DescDev D;
    D.model = d.model;
    D.n_chains = d.n_chains;
    D.unit_base = d.unit_base;
    D.flags = d.flags;
    D.seed = d.seed;
    D.max_steps = d.max_steps;
    D.n_units = desc_unit_count(d);
    D.steps = d.d_steps;
    D.perm = d.d_perm;
    D.state = d.d_state;
    D.trace = d.d_trace;
    D.trace2 = d.d_trace2;
    D.stride = d.trace_stride;
    D.offsets = d.d_offsets;
    D.ntok = d.d_ntok;
    D.step0 = 0;
    D.max_rounds = 0;
    D.progress = nullptr;
    D.unit_done = nullptr;
    D.sums = d.d_sums;
    return D;
}

brng_status launch_slots(SlotDev* slots, uint32_t n, SlotDev* tab, hipStream_t stream, int wpb) {
    if (n == 0) return BRNG_OK;
    uint32_t total = 0;
    int model = slots[0].D.model;
    int lds_wave = 0;
    for (uint32_t i = 0; i < n; ++i) {
        total += slots[i].D.n_units;
        slots[i].unit_end = total;
        slots[i].pad = 0;
        if (slots[i].D.model != model) model = M_MIXED;
        lds_wave = std::max(lds_wave, model_lds_bytes(slots[i].D.model));
    }
    if (total == 0) return BRNG_OK;
    for (uint32_t b = 0; b < n; b += PUT_CHUNK) {
        SlotChunk c;
        std::memset(&c, 0, sizeof(c));
        c.base = b;
        c.n = std::min<uint32_t>(PUT_CHUNK, n - b);
        std::memcpy(c.s, slots + b, sizeof(SlotDev) * c.n);
        hipLaunchKernelGGL(k_put_slots, dim3(1), dim3(256), 0, stream, tab, c);
    }
    while (wpb > 1 && (size_t)wpb * lds_wave > 65536) wpb >>= 1;
    const dim3 grid((total + wpb - 1) / wpb), block(64 * wpb);
    const size_t lds = (size_t)wpb * lds_wave;
    const uint32_t lw = (uint32_t)lds_wave;
    switch (model) {
        case M_TRIANGLE:
            hipLaunchKernelGGL(k_multi<M_TRIANGLE>, grid, block, lds, stream, tab, n, total, lw);
            break;
        case M_NORMEXP:
            hipLaunchKernelGGL(k_multi<M_NORMEXP>, grid, block, lds, stream, tab, n, total, lw);
            break;
        case M_GAMMA:
            hipLaunchKernelGGL(k_multi<M_GAMMA>, grid, block, lds, stream, tab, n, total, lw);
            break;
        case M_LDA:
            hipLaunchKernelGGL(k_multi<M_LDA>, grid, block, lds, stream, tab, n, total, lw);
            break;
        case M_EXPCHAIN:
            hipLaunchKernelGGL(k_multi<M_EXPCHAIN>, grid, block, lds, stream, tab, n, total, lw);
            break;
        default:
            hipLaunchKernelGGL(k_mixed, grid, block, lds, stream, tab, n, total, lw);
            break;
    }
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

}  // namespace brng

extern "C" {

const char* brng_status_string(brng_status s) {
    switch (s) {
        case BRNG_OK: return "ok";
        case BRNG_E_ARG: return "invalid argument";
        case BRNG_E_NOMEM: return "device allocation failed";
        case BRNG_E_HIP: return "HIP runtime error";
        case BRNG_E_KIND_DISABLED: return "pool kind disabled (window length 0)";
        case BRNG_E_BUSY: return "no capacity available";
        case BRNG_E_UNSUPPORTED: return "unsupported combination";
        case BRNG_E_TOO_LARGE: return "request exceeds the static scratch area";
        default: return "unknown status";
    }
}

int32_t brng_last_hip_error(void) { return g_last_hip; }

brng_status brng_create(const brng_config* cfg, brng_ctx** out) {
    if (!out) return BRNG_E_ARG;
    *out = nullptr;
    if (!cfg || cfg->n_chains == 0) return BRNG_E_ARG;
    if (cfg->layout != BRNG_LAYOUT_CHAINS && cfg->layout != BRNG_LAYOUT_ITEMS) return BRNG_E_ARG;
    if (cfg->prec != BRNG_F32 && cfg->prec != BRNG_F64) return BRNG_E_ARG;
    for (int k = 0; k < 4; ++k)
        if (!window_ok(cfg->window[k])) return BRNG_E_ARG;
    brng_ctx* c = new (std::nothrow) brng_ctx();
    if (!c) return BRNG_E_NOMEM;
    c->cfg = *cfg;
    c->stream = (hipStream_t)cfg->hip_stream;
    c->n_units = cfg->layout == BRNG_LAYOUT_CHAINS ? (cfg->n_chains + 63) / 64 : cfg->n_chains;
    c->wpb = 4;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        free_ctx(c);
        return hip_fail(e);
    }
    for (int k = 0; k < 4; ++k) {
        if (!cfg->window[k]) continue;
        const size_t bytes = (size_t)c->n_units * cfg->window[k] * kind_elem(k);
        if (hipMalloc(&c->pool[k], bytes) != hipSuccess) {
            free_ctx(c);
            return BRNG_E_NOMEM;
        }
    }
    if (hipMalloc((void**)&c->meta, sizeof(Meta) * (size_t)c->n_units) != hipSuccess ||
        hipMalloc((void**)&c->table, sizeof(SlotDev) * BRNG_BATCH_MAX) != hipSuccess ||
        hipMalloc((void**)&c->lda_plan,
                  sizeof(int32_t) * (PLAN_HEAD + PLAN_LISTS * (size_t)c->n_units)) != hipSuccess) {
        free_ctx(c);
        return BRNG_E_NOMEM;
    }
    hipLaunchKernelGGL(k_init_meta, dim3((c->n_units + 255) / 256), dim3(256), 0, c->stream,
                       c->meta, c->n_units, cfg->seed);
    e = hipGetLastError();
    if (e != hipSuccess) {
        free_ctx(c);
        return hip_fail(e);
    }
    for (int k = 0; k < 4; ++k) {
        if (!cfg->window[k]) continue;
        brng_status s = launch_fill(c, k);
        if (s != BRNG_OK) {
            free_ctx(c);
            return s;
        }
    }
    *out = c;
    return BRNG_OK;
}

brng_status brng_destroy(brng_ctx* c) {
    if (!c) return BRNG_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    free_ctx(c);
    if (e != hipSuccess) return hip_fail(e);
    return BRNG_OK;
}

brng_status brng_fill_base(brng_ctx* c, int32_t kind) {
    if (!c || kind < 0 || kind >= BRNG_NKINDS) return BRNG_E_ARG;
    if (!c->cfg.window[kind]) return BRNG_E_KIND_DISABLED;
    return launch_fill(c, kind);
}

static dim3 unit_grid(const brng_ctx* c, uint32_t n_units) {
    return dim3((n_units + c->wpb - 1) / c->wpb);
}

brng_status brng_step_uniform(brng_ctx* c, const void* a, const void* b, void* out) {
    if (!c || !a || !b || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    const int kind = c->cfg.prec == BRNG_F64 ? BRNG_U64 : BRNG_U;
    if (!c->cfg.window[kind]) return BRNG_E_KIND_DISABLED;
    const uint32_t n = c->cfg.n_chains, W = c->cfg.window[kind];
    if (kind == BRNG_U64)
        hipLaunchKernelGGL((k_step_uniform<KIND_U64, double>), unit_grid(c, c->n_units),
                           dim3(64 * c->wpb), 0, c->stream, c->meta, (double*)c->pool[kind], W, n,
                           (const double*)a, (const double*)b, (double*)out);
    else
        hipLaunchKernelGGL((k_step_uniform<KIND_U, float>), unit_grid(c, c->n_units),
                           dim3(64 * c->wpb), 0, c->stream, c->meta, (float*)c->pool[kind], W, n,
                           (const float*)a, (const float*)b, (float*)out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_normal(brng_ctx* c, const void* mu, const void* sigma, void* out) {
    if (!c || !mu || !sigma || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_N]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_normal, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_N], c->cfg.window[BRNG_N], c->cfg.n_chains,
                       (const float*)mu, (const float*)sigma, (float*)out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_exp(brng_ctx* c, const void* lam, void* out) {
    if (!c || !lam || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_E]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_exp, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_E], c->cfg.window[BRNG_E], c->cfg.n_chains,
                       (const float*)lam, (float*)out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_laplace(brng_ctx* c, const float* mu, const float* b, float* out) {
    if (!c || !mu || !b || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_E]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_laplace, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_E], c->cfg.window[BRNG_E], c->cfg.n_chains,
                       mu, b, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_weibull(brng_ctx* c, const float* lam, const float* k, float* out) {
    if (!c || !lam || !k || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_E]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_weibull, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_E], c->cfg.window[BRNG_E], c->cfg.n_chains,
                       lam, k, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_poisson(brng_ctx* c, const float* lam, int32_t* out) {
    if (!c || !lam || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_U]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_poisson, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_U], c->cfg.window[BRNG_U], c->cfg.n_chains,
                       lam, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_binomial(brng_ctx* c, const int32_t* n, const float* p, int32_t* out) {
    if (!c || !n || !p || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_U]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_binomial, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, (float*)c->pool[BRNG_U], c->cfg.window[BRNG_U], c->cfg.n_chains,
                       n, p, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_multinomial(brng_ctx* c, const int32_t* offsets, const int32_t* n,
                                  const float* w, int32_t* out) {
    if (!c || !offsets || !n || !w || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_U]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_multinomial, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0,
                       c->stream, c->meta, (float*)c->pool[BRNG_U], c->cfg.window[BRNG_U],
                       c->cfg.n_chains, offsets, n, w, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_gamma(brng_ctx* c, const float* alpha, float* out) {
    if (!c || !alpha || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_CHAINS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_N] || !c->cfg.window[BRNG_E]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_gamma, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0, c->stream,
                       c->meta, make_pools(c), c->cfg.n_chains, alpha, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_step_dirichlet(brng_ctx* c, const int32_t* offsets, const float* alpha,
                                float* out) {
    if (!c || !offsets || !alpha || !out) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_ITEMS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    if (!c->cfg.window[BRNG_N] || !c->cfg.window[BRNG_E]) return BRNG_E_KIND_DISABLED;
    hipLaunchKernelGGL(k_step_dirichlet, unit_grid(c, c->n_units), dim3(64 * c->wpb), 0,
                       c->stream, c->meta, make_pools(c), c->n_units, offsets, alpha, out);
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}


uint64_t brng_lda_full_units(uint32_t n_topics, uint32_t n_vocab, uint32_t n_docs) {
    if (n_vocab == 0) return 0;
    return (uint64_t)n_topics * ((n_vocab + LDAF_VBLOCK - 1) / LDAF_VBLOCK) + n_docs;
}

brng_status brng_run_lda_full(brng_ctx* c, const brng_lda_full_desc* d) {
    if (!c || !d) return BRNG_E_ARG;
    if (c->cfg.layout != BRNG_LAYOUT_ITEMS) return BRNG_E_ARG;
    if (c->cfg.prec != BRNG_F32) return BRNG_E_UNSUPPORTED;
    const uint32_t D = d->n_docs, K = d->n_topics, V = d->n_vocab;
    if (D == 0 || K < 1 || K > BRNG_LDAF_KMAX || V < 1 || V > BRNG_LDAF_VMAX || d->n_tokens < 0)
        return BRNG_E_ARG;
    const uint32_t nb = (V + LDAF_VBLOCK - 1) / LDAF_VBLOCK;
    if ((uint64_t)K * nb + D > c->n_units) return BRNG_E_ARG;
    if (!(d->alpha > 0.0f) || !(d->beta > 0.0f) || !std::isfinite(d->alpha) ||
        !std::isfinite(d->beta))
        return BRNG_E_ARG;
    if (!d->d_doc_offsets || !d->d_ndk || !d->d_nkw || !d->d_theta || !d->d_phi) return BRNG_E_ARG;
    if (d->n_tokens > 0 && (!d->d_words || !d->d_z)) return BRNG_E_ARG;
    if (!c->cfg.window[BRNG_U] || !c->cfg.window[BRNG_N] || !c->cfg.window[BRNG_E])
        return BRNG_E_KIND_DISABLED;
    const Pools P = make_pools(c);
    const int wpb = c->wpb;
    const dim3 blk(64 * wpb);
    // the topic blocks' gamma sums borrow the LDA planning buffer (at least
    // PLAN_LISTS n_units >= K nb words; both uses are stream-ordered)
    float* psum = reinterpret_cast<float*>(c->lda_plan);
    auto zero = [&](int32_t* p, uint64_t n) {
        const uint64_t g = std::min<uint64_t>((n + 255) / 256, 4096);
        if (g) hipLaunchKernelGGL(k_zero_i32, dim3((uint32_t)g), dim3(256), 0, c->stream, p, n);
    };
    if (d->flags & ~(uint32_t)BRNG_LDAF_COUNTS_VALID) return BRNG_E_ARG;
    if (!(d->flags & BRNG_LDAF_COUNTS_VALID)) {
        zero(d->d_ndk, (uint64_t)D * K);
        zero(d->d_nkw, (uint64_t)K * V);
        hipLaunchKernelGGL(k_ldaf_recount, dim3((D + wpb - 1) / wpb), blk, 0, c->stream, D, (int)K,
                           (int)V, d->d_doc_offsets, d->n_tokens, d->d_words, d->d_z, d->d_ndk,
                           d->d_nkw);
        HIPCHK(hipGetLastError());
    }
    // a pending event pair (brng_time_next_launch) times the last sweep's
    // document kernel
    hipEvent_t ts = c->t_start, te = c->t_stop;
    if (d->sweeps) c->t_start = c->t_stop = nullptr;
    for (uint32_t s = 0; s < d->sweeps; ++s) {
        hipLaunchKernelGGL(k_ldaf_dirichlets, dim3(K * nb + D), dim3(64), 0, c->stream, c->meta,
                           P, D, (int)K, (int)V, nb, d->alpha, d->beta, (const int32_t*)d->d_ndk,
                           (const int32_t*)d->d_nkw, d->d_theta, d->d_phi, psum);
        if (nb > 1) {
            const uint32_t g = std::min<uint32_t>(((uint32_t)K * V + 255) / 256, 2048u);
            hipLaunchKernelGGL(k_ldaf_phi_norm, dim3(g), dim3(256), 0, c->stream, (int)K, (int)V,
                               nb, (const float*)psum, d->d_phi);
        }
        zero(d->d_nkw, (uint64_t)K * V);
        if (K > 64) {
            // counts and theta per wave, K rounded up to 4 each; workgroups
            // kept within 64 KiB of LDS
            const uint32_t K4 = (K + 3) & ~3u;
            int wd = wpb;
            while (wd > 1 && (size_t)wd * 2 * K4 * sizeof(int32_t) > 65536) wd /= 2;
            const dim3 gridw((D + wd - 1) / wd), blkw(64 * wd);
            const size_t ldsw = (size_t)wd * 2 * K4 * sizeof(int32_t);
            if (ts && s + 1 == d->sweeps)
                hipExtLaunchKernelGGL(k_ldaf_docs_wide, gridw, blkw, (uint32_t)ldsw, c->stream, ts, te,
                                      0u, c->meta, P, D, (int)K, (int)V, nb, d->d_doc_offsets,
                                      d->n_tokens, d->d_words, (const float*)d->d_phi,
                                      (const float*)d->d_theta, d->d_z, d->d_ndk, d->d_nkw);
            else
                hipLaunchKernelGGL(k_ldaf_docs_wide, gridw, blkw, ldsw, c->stream, c->meta, P, D,
                                   (int)K, (int)V, nb, d->d_doc_offsets, d->n_tokens, d->d_words,
                                   (const float*)d->d_phi, (const float*)d->d_theta, d->d_z,
                                   d->d_ndk, d->d_nkw);
            HIPCHK(hipGetLastError());
            continue;
        }
        const dim3 grid((D + wpb - 1) / wpb);
        const size_t lds = (size_t)wpb * 128 * sizeof(int32_t);  // counts and theta
        auto kern = K == 16   ? k_ldaf_docs<16, true>
                    : K < 16  ? k_ldaf_docs<16, false>
                    : K == 32 ? k_ldaf_docs<32, true>
                    : K < 32  ? k_ldaf_docs<32, false>
                    : K == 64 ? k_ldaf_docs<64, true>
                              : k_ldaf_docs<64, false>;
        if (ts && s + 1 == d->sweeps)
            hipExtLaunchKernelGGL(kern, grid, blk, (uint32_t)lds, c->stream, ts, te, 0u,
                                  c->meta, P, D, (int)K, (int)V, nb, d->d_doc_offsets, d->n_tokens,
                                  d->d_words, (const float*)d->d_phi, (const float*)d->d_theta,
                                  d->d_z, d->d_ndk, d->d_nkw);
        else
            hipLaunchKernelGGL(kern, grid, blk, lds, c->stream, c->meta, P, D, (int)K,
                               (int)V, nb, d->d_doc_offsets, d->n_tokens, d->d_words,
                               (const float*)d->d_phi, (const float*)d->d_theta, d->d_z, d->d_ndk,
                               d->d_nkw);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

// A request against units [0, n_units) and windows W.
static brng_status check_desc_w(uint64_t n_units, const uint32_t* W, const brng_gibbs_desc& d) {
    if (d.model < 0 || d.model >= BRNG_NMODELS) return BRNG_E_ARG;
    if (d.n_chains == 0 || d.max_steps < 0 || !d.d_state) return BRNG_E_ARG;
    const uint64_t nu = desc_unit_count(d);
    if ((uint64_t)d.unit_base + nu > n_units) return BRNG_E_ARG;
    const int64_t width = d.model == BRNG_MODEL_LDA ? 0 : (int64_t)d.n_chains;
    if ((d.d_trace || d.d_trace2) && d.trace_stride < width) return BRNG_E_ARG;
    switch (d.model) {
        case BRNG_MODEL_TRIANGLE_F64:
            if (!W[BRNG_U64]) return BRNG_E_KIND_DISABLED;
            break;
        case BRNG_MODEL_NORMEXP:
        case BRNG_MODEL_GAMMA_CHAIN:
            if (!W[BRNG_N] || !W[BRNG_E]) return BRNG_E_KIND_DISABLED;
            break;
        case BRNG_MODEL_EXP_CHAIN:
            if (!W[BRNG_E]) return BRNG_E_KIND_DISABLED;
            break;
        case BRNG_MODEL_LDA:
            if (!d.d_offsets || !d.d_ntok) return BRNG_E_ARG;
            if (!W[BRNG_U] || !W[BRNG_N] || !W[BRNG_E]) return BRNG_E_KIND_DISABLED;
            break;
    }
    return BRNG_OK;
}

static brng_status check_desc(const brng_ctx* c, const brng_gibbs_desc& d) {
    return check_desc_w(c->n_units, c->cfg.window, d);
}


// Waves per block for a model: the requested count, halved while a block's
// LDS would exceed 64 KiB.
static int model_wpb(int wpb, int model) {
    int w = wpb;
    while (w > 1 && (size_t)w * model_lds_bytes(model) > 65536) w >>= 1;
    return w;
}

// One request's chain kernel over unit records `meta` and pools P; with an
// event pair (ts, te) the launch records them at the kernel's own start and
// end.
// plan: for LDA, PLAN_HEAD + PLAN_LISTS n_docs int32 of device memory; the
// plan kernel runs first.
static brng_status launch_gibbs(hipStream_t stream, int wpb_req, const DescDev& D, Meta* meta,
                                const Pools& P, int32_t* plan, hipEvent_t ts, hipEvent_t te) {
    const int wpb = model_wpb(wpb_req, D.model);
    const dim3 grid((D.n_units + wpb - 1) / wpb), block(64 * wpb);
    const size_t lds = (size_t)wpb * model_lds_bytes(D.model);
    if (D.model == M_LDA) {
        hipLaunchKernelGGL(k_lda_plan, dim3(1), dim3(PLAN_THREADS), 0, stream, D, plan);
        HIPCHK(hipGetLastError());
    }
#define BRNG_LAUNCH_GIBBS(MODEL)                                                               \
    do {                                                                                      \
        if (ts)                                                                               \
            hipExtLaunchKernelGGL(k_gibbs<MODEL>, grid, block, (uint32_t)lds, stream, ts, te, \
                                  0u, D, meta, P, (const int32_t*)plan);                      \
        else                                                                                  \
            hipLaunchKernelGGL(k_gibbs<MODEL>, grid, block, lds, stream, D, meta, P,          \
                               (const int32_t*)plan);                                         \
    } while (0)
    switch (D.model) {
        case M_TRIANGLE: BRNG_LAUNCH_GIBBS(M_TRIANGLE); break;
        case M_NORMEXP: BRNG_LAUNCH_GIBBS(M_NORMEXP); break;
        case M_GAMMA: BRNG_LAUNCH_GIBBS(M_GAMMA); break;
        case M_LDA:
            if (ts)
                hipExtLaunchKernelGGL(k_gibbs_lda, grid, block, (uint32_t)lds, stream, ts, te, 0u,
                                      D, meta, P, (const int32_t*)plan);
            else
                hipLaunchKernelGGL(k_gibbs_lda, grid, block, lds, stream, D, meta, P,
                                   (const int32_t*)plan);
            break;
        default: BRNG_LAUNCH_GIBBS(M_EXPCHAIN); break;
    }
#undef BRNG_LAUNCH_GIBBS
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

static brng_status launch_plain(brng_ctx* c, const DescDev& D) {
    // a pending event pair is used by this launch, then forgotten
    hipEvent_t ts = c->t_start, te = c->t_stop;
    c->t_start = c->t_stop = nullptr;
    return launch_gibbs(c->stream, c->wpb, D, c->meta, make_pools(c), c->lda_plan, ts, te);
}


// Batched form: all requests in one launch, in the order given (the mixed
// kernel when their models differ).
static brng_status launch_batched(brng_ctx* c, const brng_gibbs_desc* descs, uint32_t n_desc) {
    const Pools P = make_pools(c);
    std::vector<SlotDev> S(n_desc);
    for (uint32_t i = 0; i < n_desc; ++i) {
        S[i].D = desc_to_device(descs[i]);
        S[i].meta = c->meta;
        S[i].P = P;
    }
    return launch_slots(S.data(), n_desc, c->table, c->stream, c->wpb);
}

brng_status brng_run_gibbs(brng_ctx* c, const brng_gibbs_desc* descs, uint32_t n_desc) {
    if (!c || !descs || n_desc == 0 || n_desc > BRNG_BATCH_MAX) return BRNG_E_ARG;
    for (uint32_t i = 0; i < n_desc; ++i) {
        brng_status s = check_desc(c, descs[i]);
        if (s != BRNG_OK) return s;
    }
    // requests must not share units
    std::vector<std::pair<uint32_t, uint32_t>> ranges(n_desc);
    for (uint32_t i = 0; i < n_desc; ++i)
        ranges[i] = {descs[i].unit_base, descs[i].unit_base + desc_unit_count(descs[i])};
    std::sort(ranges.begin(), ranges.end());
    for (uint32_t i = 1; i < n_desc; ++i)
        if (ranges[i].first < ranges[i - 1].second) return BRNG_E_ARG;
    if (n_desc == 1) return launch_plain(c, desc_to_device(descs[0]));
    // several requests (independent: their units are disjoint) share launches
    return launch_batched(c, descs, n_desc);
}

// ---------------------------------------------------------------------------
// Chain runs without allocation: the unit records and pool windows of the
// request live in one file-scope device array of fixed size, which each GPU
// holds until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr uint64_t STATIC_SCRATCH_BYTES = (uint64_t)BRNG_STATIC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES];

// Address of this device's scratch array, looked up once per device with
// that device current.
static brng_status scratch_address(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return BRNG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return BRNG_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BRNG_OK;
}

static uint64_t scratch_round(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

brng_status brng_run_gibbs_static(const brng_gibbs_desc* d, const uint32_t* window4, int32_t wpb,
                                  void* stream) {
    if (!d || !window4) return BRNG_E_ARG;
    if (!(wpb == 1 || wpb == 2 || wpb == 4 || wpb == 8)) return BRNG_E_ARG;
    for (int k = 0; k < 4; ++k)
        if (!window_ok(window4[k])) return BRNG_E_ARG;
    // a fresh request on request-local units 0..n_units-1
    if (d->unit_base != 0 || (d->flags & BRNG_FLAG_RESUME) || d->flags != 0) return BRNG_E_ARG;
    const uint64_t nu = desc_unit_count(*d);
    brng_status st = check_desc_w(nu, window4, *d);
    if (st != BRNG_OK) return st;
    // the kinds the model reads, each n_units windows; then the unit records
    bool need[4] = {false, false, false, false};
    switch (d->model) {
        case BRNG_MODEL_TRIANGLE_F64: need[BRNG_U64] = true; break;
        case BRNG_MODEL_NORMEXP:
        case BRNG_MODEL_GAMMA_CHAIN: need[BRNG_N] = need[BRNG_E] = true; break;
        case BRNG_MODEL_EXP_CHAIN: need[BRNG_E] = true; break;
        default: need[BRNG_U] = need[BRNG_N] = need[BRNG_E] = true; break;
    }
    uint64_t off[4] = {0, 0, 0, 0}, total = 0;
    for (int k = 0; k < 4; ++k) {
        if (!need[k]) continue;
        off[k] = total;
        total += scratch_round(nu * window4[k] * kind_elem(k));
    }
    const uint64_t meta_off = total;
    total += scratch_round(nu * sizeof(Meta));
    const uint64_t plan_off = total;  // LDA: the launch plan and its scratch
    if (d->model == BRNG_MODEL_LDA)
        total += scratch_round((PLAN_HEAD + PLAN_LISTS * nu) * sizeof(int32_t));
    if (total > STATIC_SCRATCH_BYTES) return BRNG_E_TOO_LARGE;
    void* base = nullptr;
    st = scratch_address(&base);
    if (st != BRNG_OK) return st;
    char* b = static_cast<char*>(base);
    Pools P;
    P.u = need[BRNG_U] ? reinterpret_cast<float*>(b + off[BRNG_U]) : nullptr;
    P.n = need[BRNG_N] ? reinterpret_cast<float*>(b + off[BRNG_N]) : nullptr;
    P.e = need[BRNG_E] ? reinterpret_cast<float*>(b + off[BRNG_E]) : nullptr;
    P.u64 = need[BRNG_U64] ? reinterpret_cast<double*>(b + off[BRNG_U64]) : nullptr;
    for (int k = 0; k < 4; ++k) P.W[k] = need[k] ? window4[k] : 0;
    // a fresh request reads nothing of the array before writing it: its
    // windows start empty (regenerated on first use) and its unit records
    // are built in registers and written at the end
    return launch_gibbs((hipStream_t)stream, wpb, desc_to_device(*d),
                        reinterpret_cast<Meta*>(b + meta_off), P,
                        reinterpret_cast<int32_t*>(b + plan_off), nullptr, nullptr);
}

brng_status brng_sort_by_length(uint32_t n, const int32_t* steps, int32_t* perm) {
    if ((n && (!steps || !perm))) return BRNG_E_ARG;
    std::vector<int32_t> idx(n);
    for (uint32_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int32_t a, int32_t b) { return steps[a] > steps[b]; });
    std::memcpy(perm, idx.data(), sizeof(int32_t) * n);
    return BRNG_OK;
}

brng_status brng_get_cursors(brng_ctx* c, uint64_t* out) {
    if (!c || !out) return BRNG_E_ARG;
    uint64_t* d = nullptr;
    const size_t bytes = sizeof(uint64_t) * 4 * (size_t)c->n_units;
    HIPCHK(hipMalloc(&d, bytes));
    hipLaunchKernelGGL(k_get_cursors, dim3((c->n_units + 255) / 256), dim3(256), 0, c->stream,
                       c->meta, c->n_units, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e);
    return BRNG_OK;
}

brng_status brng_set_cursors(brng_ctx* c, const uint64_t* in) {
    if (!c || !in) return BRNG_E_ARG;
    uint64_t* d = nullptr;
    const size_t bytes = sizeof(uint64_t) * 4 * (size_t)c->n_units;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMalloc(&d, bytes));
    hipError_t e = hipMemcpy(d, in, bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_set_cursors, dim3((c->n_units + 255) / 256), dim3(256), 0,
                           c->stream, c->meta, c->n_units, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e);
    return BRNG_OK;
}

brng_status brng_get_window(brng_ctx* c, int32_t kind, uint32_t unit, void* out, uint32_t cap,
                            uint64_t* base, uint32_t* len) {
    if (!c || kind < 0 || kind >= BRNG_NKINDS || unit >= c->n_units || !base || !len)
        return BRNG_E_ARG;
    if (!c->cfg.window[kind]) return BRNG_E_KIND_DISABLED;
    Meta m;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(&m, c->meta + unit, sizeof(Meta), hipMemcpyDeviceToHost));
    *base = m.wbase[kind];
    *len = m.wlen[kind];
    const uint32_t n = std::min(cap, c->cfg.window[kind]);
    if (n && out) {
        const size_t el = kind_elem(kind);
        const char* src = (const char*)c->pool[kind] + (size_t)unit * c->cfg.window[kind] * el;
        HIPCHK(hipMemcpy(out, src, n * el, hipMemcpyDeviceToHost));
    }
    return BRNG_OK;
}

brng_status brng_convert(int32_t kind, const uint32_t* words, uint64_t n_words, void* out,
                         void* stream) {
    if (kind < 0 || kind >= BRNG_NKINDS || (n_words & 3) || (n_words && (!words || !out)))
        return BRNG_E_ARG;
    if (((uintptr_t)words & 15) || ((uintptr_t)out & 15)) return BRNG_E_ARG;
    const uint64_t nblk = n_words / 4;
    if (!nblk) return BRNG_OK;
    const dim3 grid((unsigned)((nblk + 255) / 256));
    hipStream_t st = (hipStream_t)stream;
    const uint4* w = (const uint4*)words;
    uint4* o = (uint4*)out;
    switch (kind) {
        case BRNG_U: hipLaunchKernelGGL(k_convert<KIND_U>, grid, dim3(256), 0, st, w, nblk, o); break;
        case BRNG_N: hipLaunchKernelGGL(k_convert<KIND_N>, grid, dim3(256), 0, st, w, nblk, o); break;
        case BRNG_E: hipLaunchKernelGGL(k_convert<KIND_E>, grid, dim3(256), 0, st, w, nblk, o); break;
        default: hipLaunchKernelGGL(k_convert<KIND_U64>, grid, dim3(256), 0, st, w, nblk, o); break;
    }
    HIPCHK(hipGetLastError());
    return BRNG_OK;
}

brng_status brng_get_info(const brng_ctx* c, uint32_t* n_units, uint32_t* window4) {
    if (!c) return BRNG_E_ARG;
    if (n_units) *n_units = c->n_units;
    if (window4)
        for (int k = 0; k < 4; ++k) window4[k] = c->cfg.window[k];
    return BRNG_OK;
}

brng_status brng_set_launch(brng_ctx* c, int32_t wpb, int32_t reserved) {
    if (!c || !(wpb == 1 || wpb == 2 || wpb == 4 || wpb == 8) || reserved != 0) return BRNG_E_ARG;
    c->wpb = wpb;
    return BRNG_OK;
}

brng_status brng_time_next_launch(brng_ctx* c, void* start_event, void* stop_event) {
    if (!c || (start_event == nullptr) != (stop_event == nullptr)) return BRNG_E_ARG;
    c->t_start = static_cast<hipEvent_t>(start_event);
    c->t_stop = static_cast<hipEvent_t>(stop_event);
    return BRNG_OK;
}

}  // extern "C"
