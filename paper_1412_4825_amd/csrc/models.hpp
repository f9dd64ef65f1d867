// Chain models: many independent Gibbs chains, one wave per unit of 64
// chains (or one document), state in registers for every step of the run.
//
// The paper's example (Eq. 1, Fig. 1) alternates x ~ U(0, 1-y) and
// y ~ U(0, 1-x); its motivating application (Sec. 1, LDA) redraws a
// Dirichlet whose parameters change every sweep.  Every model below is one
// loop over steps; each step is a fixed sequence of pool calls (one entry
// per active lane, lanes in order), so the consumed entries, and with them
// every output, are fixed by the seed alone.
#pragma once
#include "samplers.hpp"

namespace brng {

// Device copy of one request (brng_gibbs_desc plus derived fields).
struct DescDev {
    int32_t model;
    uint32_t n_chains;
    uint32_t unit_base;
    uint32_t flags;
    uint64_t seed;
    int32_t max_steps;
    uint32_t n_units;
    const int32_t* steps;
    const int32_t* perm;
    void* state;
    void* trace;
    void* trace2;
    int64_t stride;
    const int32_t* offsets;
    const int32_t* ntok;
    uint32_t queue_first;  // first index of this request in the batched queue
    uint32_t pad;
};

enum : int32_t { M_TRIANGLE = 0, M_NORMEXP = 1, M_GAMMA = 2, M_LDA = 3, M_EXPCHAIN = 4 };
enum : uint32_t { FLAG_RESUME = 1u };

// Per-wave LDS: three rings and an auxiliary area (LDA bin boundaries and
// counts).
constexpr int AUX_BYTES = 2048;
constexpr int WAVE_LDS_BYTES = 3 * RING_BYTES + AUX_BYTES;

struct Pools {
    float* u;
    float* n;
    float* e;
    double* u64;
    uint32_t W[4];
};

// A fresh request starts its unit's streams at index 0 with empty windows;
// the record is built in registers and its key written back at the end.
__device__ __forceinline__ Meta fresh_meta(const DescDev& D, uint32_t local) {
    Meta m;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m.cur[k] = 0;
        m.wbase[k] = 0;
        m.wlen[k] = 0;
    }
    m.key_unit = local;
    m.pad = 0;
    m.key_seed = D.seed;
    return m;
}

__device__ __forceinline__ Meta open_meta(const DescDev& D, const Meta* mp, uint32_t local) {
    if (D.flags & FLAG_RESUME) return *mp;
    return fresh_meta(D, local);
}

__device__ __forceinline__ void store_key(Meta* mp, const Meta& m) {
    if (lane_id() == 0) {
        mp->key_unit = m.key_unit;
        mp->key_seed = m.key_seed;
    }
}

// ---------------------------------------------------------------------------
// Triangle (Eq. 1, Fig. 1) in fp64: x <- (1 - y) u then y <- (1 - x) u',
// u, u' from the U64 pool.  The products and differences are rounded one at
// a time (no fused multiply-add), as in the reference definition, so the
// trajectories match bit for bit.
// ---------------------------------------------------------------------------
__device__ void unit_triangle(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                              unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot = local * 64 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;  // a bad permutation entry idles the lane
    const int32_t L = in ? (D.steps ? D.steps[chain] : D.max_steps) : 0;
    const Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    StagedReader<KIND_U64> ru;
    ru.open(m, P.u64 + (size_t)gu * P.W[KIND_U64], P.W[KIND_U64], reinterpret_cast<double*>(lds));
    double* st = reinterpret_cast<double*>(D.state);
    double x = 0.5, y = 0.5;
    if ((D.flags & FLAG_RESUME) && in) {
        x = st[chain];
        y = st[(size_t)D.n_chains + chain];
    }
    double* tx = reinterpret_cast<double*>(D.trace);
    double* ty = reinterpret_cast<double*>(D.trace2);
    const int32_t smax = D.max_steps;
    for (int32_t t = 0; t < smax; ++t) {
        const bool act = in && t < L;
        if (wave_ballot(act) == 0) break;
        const double u1 = ru.take(act);
        if (act) x = __dmul_rn(__dsub_rn(1.0, y), u1);
        const double u2 = ru.take(act);
        if (act) y = __dmul_rn(__dsub_rn(1.0, x), u2);
        if (act) {
            if (tx) tx[(size_t)t * D.stride + slot] = x;
            if (ty) ty[(size_t)t * D.stride + slot] = y;
        }
    }
    if (in) {
        st[chain] = x;
        st[(size_t)D.n_chains + chain] = y;
    }
    ru.close(*mp);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Normal/exponential chain: s' = 0.9 s + (0.5 + |s|) z, e = E / (1 + s'^2).
// Fresh chains draw s_0 as their first Gaussian.
// ---------------------------------------------------------------------------
__device__ void unit_normexp(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                             unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot = local * 64 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;  // a bad permutation entry idles the lane
    const int32_t L = in ? (D.steps ? D.steps[chain] : D.max_steps) : 0;
    const bool fresh = !(D.flags & FLAG_RESUME);
    const Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    StagedReader<KIND_N> rn;
    StagedReader<KIND_E> re;
    rn.open(m, P.n + (size_t)gu * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + RING_BYTES));
    float* st = reinterpret_cast<float*>(D.state);
    float s;
    if (fresh)
        s = rn.take(in);
    else
        s = in ? st[chain] : 0.0f;
    float* ts = reinterpret_cast<float*>(D.trace);
    float* te = reinterpret_cast<float*>(D.trace2);
    const int32_t smax = D.max_steps;
    const bool full = (wave_ballot(in && L >= smax) == ~0ull);
    if (full && ts && te) {
        // every lane runs every step: no ballots, four steps per ring check
        int32_t t = 0;
        for (; t + 4 <= smax; t += 4) {
            rn.ensure(rn.cur + 256);
            re.ensure(re.cur + 256);
            float z[4], ee[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z[i] = rn.ring[(rn.cur + 64 * i + lane) & (rn.R - 1)];
                ee[i] = re.ring[(re.cur + 64 * i + lane) & (re.R - 1)];
            }
            rn.cur += 256;
            re.cur += 256;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float sp = fmaf(0.5f + fabsf(s), z[i], 0.9f * s);
                const float lam = fmaf(sp, sp, 1.0f);
                ts[(size_t)(t + i) * D.stride + slot] = sp;
                te[(size_t)(t + i) * D.stride + slot] = ee[i] / lam;
                s = sp;
            }
        }
        for (; t < smax; ++t) {
            const float z = rn.take_all();
            const float sp = fmaf(0.5f + fabsf(s), z, 0.9f * s);
            const float e = re.take_all();
            ts[(size_t)t * D.stride + slot] = sp;
            te[(size_t)t * D.stride + slot] = e / fmaf(sp, sp, 1.0f);
            s = sp;
        }
    } else {
        for (int32_t t = 0; t < smax; ++t) {
            const bool act = in && t < L;
            if (wave_ballot(act) == 0) break;
            const float z = rn.take(act);
            const float sp = fmaf(0.5f + fabsf(s), z, 0.9f * s);
            const float e = re.take(act);
            if (act) {
                if (ts) ts[(size_t)t * D.stride + slot] = sp;
                if (te) te[(size_t)t * D.stride + slot] = e / fmaf(sp, sp, 1.0f);
                s = sp;
            }
        }
    }
    if (in) st[chain] = s;
    rn.close(*mp);
    re.close(*mp);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Exponential chain (served form's exponential kind): e' = E / (1 + e^2).
// Fresh chains draw e_0 as their first exponential.
// ---------------------------------------------------------------------------
__device__ void unit_expchain(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                              unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot = local * 64 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;  // a bad permutation entry idles the lane
    const int32_t L = in ? (D.steps ? D.steps[chain] : D.max_steps) : 0;
    const bool fresh = !(D.flags & FLAG_RESUME);
    const Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    StagedReader<KIND_E> re;
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E], reinterpret_cast<float*>(lds));
    float* st = reinterpret_cast<float*>(D.state);
    float v;
    if (fresh)
        v = re.take(in);
    else
        v = in ? st[chain] : 0.0f;
    float* tr = reinterpret_cast<float*>(D.trace);
    for (int32_t t = 0; t < D.max_steps; ++t) {
        const bool act = in && t < L;
        if (wave_ballot(act) == 0) break;
        const float e = re.take(act);
        if (act) {
            v = e / fmaf(v, v, 1.0f);
            if (tr) tr[(size_t)t * D.stride + slot] = v;
        }
    }
    if (in) st[chain] = v;
    re.close(*mp);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Varying-shape gamma chain: g_t ~ Gamma(alpha_t, 1), alpha_{t+1} = 0.1 + g_t.
// ---------------------------------------------------------------------------
__device__ void unit_gamma(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                           unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot = local * 64 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;  // a bad permutation entry idles the lane
    const int32_t L = in ? (D.steps ? D.steps[chain] : D.max_steps) : 0;
    const Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    StagedReader<KIND_N> rn;
    StagedReader<KIND_E> re;
    rn.open(m, P.n + (size_t)gu * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + RING_BYTES));
    float* st = reinterpret_cast<float*>(D.state);
    float alpha = in ? st[chain] : 1.0f;
    float* tg = reinterpret_cast<float*>(D.trace);
    for (int32_t t = 0; t < D.max_steps; ++t) {
        const bool act = in && t < L;
        if (wave_ballot(act) == 0) break;
        const float g = gamma_call(rn, re, act, alpha);
        if (act) {
            if (tg) tg[(size_t)t * D.stride + slot] = g;
            alpha = 0.1f + g;
        }
    }
    if (in) st[chain] = alpha;
    rn.close(*mp);
    re.close(*mp);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Dirichlet for one item of K components (batches of 64 lanes, one gamma
// call per batch, ascending), normalised by the sum (Sec. 1, footnote).
// y holds up to 4 batches (K <= 256) in registers; larger K reads alpha per
// batch and keeps y in the output array.
// ---------------------------------------------------------------------------
constexpr int LDA_KMAX = 256;

template <class RN, class RE>
__device__ __forceinline__ float dirichlet_sum4(RN& rn, RE& re, int K, const float* alpha_of,
                                                float y[4]) {
    const uint32_t lane = lane_id();
    float part = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int k = b * 64 + (int)lane;
        if (b * 64 < K) {
            const bool act = k < K;
            y[b] = gamma_call(rn, re, act, act ? alpha_of[b] : 1.0f);
            if (act) part += y[b];
        } else {
            y[b] = 0.0f;
        }
    }
    return wave_sum(part);
}

// ---------------------------------------------------------------------------
// LDA-style document: per sweep, theta ~ Dirichlet(0.1 + counts), then
// counts ~ Multinomial(n, theta) by the integer-exact rule:
//   q_k = rint(theta_k 2^24), Q = sum q_k (all q_k = 1 when Q = 0),
//   C_k = q_0 + ... + q_k; token i takes u_i from the U pool,
//   j = (u_i 2^24 - 1) / 2, t = (j Q) >> 23, bin = first k with t < C_k.
// ---------------------------------------------------------------------------
__device__ void unit_lda(const DescDev& D, Meta* mp, const Pools& P, uint32_t doc,
                         unsigned char* lds) {
    const uint32_t lane = lane_id();
    const Meta m = open_meta(D, mp, doc);
    const uint32_t gu = D.unit_base + doc;
    const int32_t off = D.offsets[doc];
    const int K = D.offsets[doc + 1] - off;
    const int ntok = D.ntok[doc];
    StagedReader<KIND_N> rn;
    StagedReader<KIND_E> re;
    StagedReader<KIND_U> ru;
    rn.open(m, P.n + (size_t)gu * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + RING_BYTES));
    ru.open(m, P.u + (size_t)gu * P.W[KIND_U], P.W[KIND_U],
            reinterpret_cast<float*>(lds + 2 * RING_BYTES));
    int32_t* Cs = reinterpret_cast<int32_t*>(lds + 3 * RING_BYTES);  // 256 bin ends
    int32_t* cnt = Cs + LDA_KMAX;                                      // 256 counts
    int32_t* counts = reinterpret_cast<int32_t*>(D.state) + off;
    float* th_tr = reinterpret_cast<float*>(D.trace);
    int32_t* ct_tr = reinterpret_cast<int32_t*>(D.trace2);
    int32_t c[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int k = b * 64 + (int)lane;
        c[b] = (k < K) ? counts[k] : 0;
    }
    for (int32_t sw = 0; sw < D.max_steps; ++sw) {
        float al[4], y[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) al[b] = 0.1f + (float)c[b];
        const float S = dirichlet_sum4(rn, re, K, al, y);
        // theta, quantised weights and their prefix sums
        int32_t carry = 0;
        float th[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (b * 64 < K) {
                th[b] = (k < K && S > 0.0f) ? y[b] / S : 0.0f;
                const int32_t q = (k < K) ? (int32_t)rintf(th[b] * 16777216.0f) : 0;
                const int32_t inc = wave_incl_scan(q) + carry;
                if (k < K) Cs[k] = inc;
                carry = __shfl(inc, 63, 64);
            } else {
                th[b] = 0.0f;
            }
        }
        int32_t Q = carry;
        if (Q == 0) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = b * 64 + (int)lane;
                if (k < K) Cs[k] = k + 1;
            }
            Q = K;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (k < K) cnt[k] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int i0 = 0; i0 < ntok; i0 += 64) {
            const bool act = i0 + (int)lane < ntok;
            const float u = ru.take(act);
            if (act) {
                const uint32_t j = ((uint32_t)(u * 16777216.0f) - 1u) >> 1;
                const uint32_t t = (uint32_t)(((uint64_t)j * (uint32_t)Q) >> 23);
                int lo = 0, hi = K - 1;  // first k with t < Cs[k]
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((uint32_t)Cs[mid] > t)
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                atomicAdd(&cnt[lo], 1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (k < K) {
                c[b] = cnt[k];
                if (th_tr) th_tr[(size_t)sw * D.stride + off + k] = th[b];
                if (ct_tr) ct_tr[(size_t)sw * D.stride + off + k] = c[b];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int k = b * 64 + (int)lane;
        if (k < K) counts[k] = c[b];
    }
    rn.close(*mp);
    re.close(*mp);
    ru.close(*mp);
    store_key(mp, m);
}

}  // namespace brng
