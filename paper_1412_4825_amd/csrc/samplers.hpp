// Samplers built on the pools: the reducible transforms of Sec. 2.1 and the
// irreducible gamma (Sec. 2.2, GetGamma) with Dirichlet on top of it (Sec. 1,
// footnote on Dirichlet).
//
// Gamma follows Marsaglia & Tsang (ACM TOMS 26(3), 2000): for shape a >= 1,
// d = a - 1/3, c = 1/sqrt(9d); draw x ~ N(0,1) until v0 = 1 + c x > 0, then
// accept d v0^3 when ln u < x^2/2 + d (1 - v + ln v), v = v0^3.  ln u is -E
// for an entry E of the exponential pool (the paper's log-uniform buffer).
// For a < 1 the draw is made at a + 1 and multiplied by u'^(1/a), taken as
// exp(-E'/a) with E' from the exponential pool.
//
// Writing y = c x, the accept statistic x^2/2 + d (1 - v + ln v) equals
// d q(y) with q(y) = 3 ln(1+y) - 3y + 3y^2/2 - y^3.  In fp32 q loses digits
// to cancellation, so the wave decides in fp32 only when the statistic is
// clear of its fp32 error bound and otherwise recomputes it in fp64.
#pragma once
#include "pool.hpp"

namespace brng {

// q(y) in double precision: a power series near 0 (q = sum_{k>=4}
// 3 (-1)^(k+1) y^k / k), the closed form elsewhere.
__device__ __noinline__ double mt_q64(double y) {
    if (fabs(y) < 0.125) {
        // 18 terms: |y|^18 / 21 < 2^-56 for |y| < 1/8.
        double p = 0.0;
#pragma unroll
        for (int k = 21; k >= 4; --k) {
            const double coef = ((k & 1) ? 3.0 : -3.0) / (double)k;
            p = fma(p, y, coef);
        }
        const double y2 = y * y;
        return p * y2 * y2;
    }
    return 3.0 * log1p(y) - 3.0 * y + 1.5 * y * y - y * y * y;
}

// Accept statistic E + d q(y) in fp64 from the fp32 inputs.
__device__ __noinline__ bool mt_accept64(float a, float x, float e) {
    const double d = (double)a - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    const double y = c * (double)x;
    return (double)e + d * mt_q64(y) > 0.0;
}

// Shapes outside (0, 2^64) would never be accepted (or are meaningless);
// such draws complete at once with NaN and consume nothing.
__device__ __forceinline__ bool gamma_shape_ok(float alpha) {
    return alpha > 0.0f && alpha < 0x1p64f;
}

// Per-lane constants of the draw a lane holds.
struct GammaLane {
    float alpha, a, d, c;
    bool valid, boost;
    __device__ __forceinline__ void setup(float al) {
        alpha = al;
        valid = gamma_shape_ok(al);
        boost = valid && al < 1.0f;
        a = valid ? (boost ? al + 1.0f : al) : 1.0f;
        d = a - (1.0f / 3.0f);
        c = __builtin_amdgcn_rsqf(9.0f * d);  // 1 / sqrt(9 d)
    }
};

// ln(1 + y) for y > -1: the logarithm of the rounded sum u = 1 + y plus the
// first-order correction for the rounding (y - (u - 1)) / u.
__device__ __forceinline__ float log1p_fast(float y) {
    const float u = 1.0f + y;
    const float corr = (y - (u - 1.0f)) * __builtin_amdgcn_rcpf(u);
    return fmaf(__builtin_amdgcn_logf(u), 0.693147180559945309f, corr);
}

// The accept statistic E + d q(y) in fp32 for a lane with 1 + c x = v0 > 0:
// *acc is its sign, *unsure whether it lies within its fp32 error bound of
// zero (term magnitudes times a few ulp, plus the effect of y's own
// rounding), in which case the decision is taken again in fp64.
__device__ __forceinline__ void mt_test(float d, float y, float v0, float e, bool* acc,
                                        bool* unsure) {
    const float l = log1p_fast(y);
    const float y2 = y * y;
    const float y3 = y2 * y;
    const float q = (3.0f * l - 3.0f * y) + (1.5f * y2 - y3);
    const float stat = e + d * q;
    const float mag = e + d * (3.0f * fabsf(l) + 3.0f * fabsf(y) + 1.5f * y2 + fabsf(y3) +
                               3.0f * y2 * y2 * __builtin_amdgcn_rcpf(v0));
    *acc = stat > 0.0f;
    *unsure = !(fabsf(stat) > 2e-6f * mag);
}

// Gamma draws in rounds over the 64 lanes of a wave.  Each lane holds at most
// one draw.  Per round: a Gaussian for every lane holding a valid draw, an
// exponential for those with 1 + c x > 0, the accept test, an exponential for
// accepted draws with alpha < 1 (the boost), each call handing entries to
// lanes in lane order; then every lane whose draw is complete hands its value
// to the source and takes its next draw.  Every EPOCH_ROUNDS rounds the
// readers stage their next chunks and the source flushes what it buffered
// (the readers' epoch points).
//
// The loop carries only numbers (the shape of the draw each lane holds and
// the source's counters); the per-lane conditions are derived from them at
// the top of each round, which keeps lane-mask bookkeeping out of the loop.
// Src provides:
//   float first()                 shape of this lane's first draw (any
//                                 value if it holds none)
//   bool holding()                whether this lane holds a draw
//   float complete(bool done, float g, float alpha)
//                                 called by every lane; a lane whose draw is
//                                 done hands over g; returns the shape of the
//                                 lane's draw for the next round
//   void flush()                  epoch point (global stores go here)
constexpr uint32_t EPOCH_ROUNDS = 4;

// COVERED: the readers' rings hold an epoch's worst case (64 Gaussians and
// 128 exponentials per round), so no call inside the rounds needs to stage.
template <bool COVERED, class RN, class RE, class Src>
__device__ __forceinline__ void gamma_rounds(RN& rn, RE& re, Src& src, uint32_t max_rounds) {
    float al = src.first();
    // Let every load issued so far land here, once: otherwise the first use
    // of a loaded value inside the loop makes the compiler wait for all
    // memory operations in flight at that point of every round.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    for (uint32_t round = 0; round < max_rounds; ++round) {
        const bool hold = src.holding();
        if (wave_ballot(hold) == 0) break;
        if ((round & (EPOCH_ROUNDS - 1)) == 0) {
            epoch_point(rn, re);
            src.flush();
        }
        GammaLane L;
        L.setup(al);
        const bool pend = hold && L.valid;
        // The Gaussian call and the exponential call hand entries to the
        // same lanes whenever every pending lane has 1 + c x > 0, which is
        // nearly always: both are read with the same ranks at once, and the
        // exponential call is redone with its own ranks when it is not so.
        const uint64_t mp = wave_ballot(pend);
        const uint32_t np = (uint32_t)__popcll(mp);
        if (!COVERED) {
            rn.reserve(np);
            re.reserve(np);
        }
        const uint32_t rk = mask_rank(mp);
        const float xr = rn.peek(rk);
        float e = re.peek(rk);
        rn.advance(np);
        const float x = pend ? xr : 0.0f;
        const float y = L.c * x;
        const float v0 = 1.0f + y;
        const bool need_e = pend && v0 > 0.0f;
        const uint64_t me = wave_ballot(need_e);
        if (me == mp) {
            re.advance(np);
        } else {
            e = re.peek(mask_rank(me));
            re.advance((uint32_t)__popcll(me));
        }
        // One lane in twenty-odd needs the logarithm in a round, so the wave
        // nearly always does: every lane evaluates the test, and only lanes
        // whose fp32 statistic is within its error bound of zero (rare)
        // decide again in fp64.
        bool acc, unsure;
        mt_test(L.d, y, v0, e, &acc, &unsure);
        acc = need_e && acc;
        unsure = need_e && unsure;
        if (wave_ballot(unsure) != 0) {
            if (unsure) acc = mt_accept64(L.a, x, e);
        }
        float g = L.d * (v0 * v0 * v0);
        const bool b = acc && L.boost;
        // boost: g exp(-E'/alpha) = 2^(log2 g - E' log2(e) / alpha), one
        // exponential whose result underflows only when the product does
        const uint64_t mb = wave_ballot(b);
        if (mb != 0) {
            const uint32_t nb = (uint32_t)__popcll(mb);
            if (!COVERED) re.reserve(nb);
            const float e2 = re.peek(mask_rank(mb));
            re.advance(nb);
            const float gb = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(g) -
                                                    e2 * (1.44269504088896341f * __builtin_amdgcn_rcpf(al)));
            g = b ? gb : g;
        }
        const bool done = hold && (acc || !L.valid);
        g = L.valid ? g : __builtin_nanf("");
        al = src.complete(done, g, al);
    }
    src.flush();
}

// One draw per lane (the one-at-a-time call).
struct OneEachSrc {
    int32_t want;  // 1 while this lane's draw is pending
    float alpha;
    float g;
    __device__ __forceinline__ float first() { return want ? alpha : 1.0f; }
    __device__ __forceinline__ bool holding() const { return want != 0; }
    __device__ __forceinline__ float complete(bool done, float gv, float al) {
        g = done ? gv : g;
        want = done ? 0 : want;
        return al;
    }
    __device__ __forceinline__ void flush() {}
};

// Components of one Dirichlet item: lanes start with components 0..63 and a
// lane whose draw completes takes the lowest component not yet started.
// y receives component k's gamma at y[k].
struct CompSrc {
    int K;
    uint32_t next;  // wave-uniform
    int comp;
    const float* alpha;  // per component, or null: 0.1 + cnt[k]
    const int32_t* cnt;
    float* y;
    __device__ __forceinline__ float shape(int k) const {
        return alpha ? alpha[k] : 0.1f + (float)cnt[k];
    }
    __device__ __forceinline__ float first() {
        comp = (int)lane_id();
        next = (uint32_t)min(K, 64);
        return comp < K ? shape(comp) : 1.0f;
    }
    __device__ __forceinline__ bool holding() const { return comp < K; }
    __device__ __forceinline__ float complete(bool done, float gv, float al) {
        if (done) y[comp] = gv;
        const uint64_t freed = wave_ballot(done);
        const uint32_t r = mask_rank(freed);
        float a = al;
        if (done) {
            comp = (int)(next + r);
            if (comp < K) a = shape(comp);
        }
        next += (uint32_t)__popcll(freed);
        return a;
    }
    __device__ __forceinline__ void flush() {}
};

// One chain per lane: g_t ~ Gamma(alpha_t, 1), alpha_{t+1} = 0.1 + g_t; the
// lane starts its next step as soon as a draw is accepted.  Trace values wait
// in LDS (at most EPOCH_ROUNDS per lane, one per round) and go out at the
// epoch points.
struct ChainSrc {
    int32_t t, L;
    float alpha;
    bool trace;      // wave-uniform: write the trace
    float* out;      // this lane's entry of the trace row of the next flushed step
    int64_t stride;  // trace elements between steps
    float* obuf;     // LDS, EPOCH_ROUNDS x 64 values; this lane's column
    uint32_t nb;     // values buffered by this lane
    __device__ __forceinline__ float first() {
        nb = 0;
        return alpha;
    }
    __device__ __forceinline__ bool holding() const { return t < L; }
    // Branch-free: every lane writes its value to its next buffer slot, and
    // only lanes whose draw completed move on (a slot written by a lane that
    // did not is overwritten before it is flushed).
    __device__ __forceinline__ float complete(bool done, float gv, float) {
        if (trace) {
            obuf[nb * 64] = gv;
            nb += done ? 1u : 0u;
        }
        alpha = done ? 0.1f + gv : alpha;
        t += done ? 1 : 0;
        return alpha;
    }
    __device__ __forceinline__ void flush() {
        if (trace) {
            static_for<0, (int)EPOCH_ROUNDS>([&](auto jc) {
                constexpr uint32_t j = decltype(jc)::value;
                if (j < nb) {
                    *out = obuf[j * 64];
                    out += stride;
                }
            });
        }
        nb = 0;
    }
};

// Sum over the wave, identical in every lane (fixed butterfly order, then
// lane 0's value broadcast).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
}

// Inclusive prefix sum over lanes (integers, exact).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

}  // namespace brng
