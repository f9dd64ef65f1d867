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
#include <type_traits>

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

// ln(1 + y) for y > -1: the logarithm of the rounded sum u = 1 + y plus the
// first-order correction for the rounding (y - (u - 1)) / u.
__device__ __forceinline__ float log1p_fast(float y) {
    const float u = 1.0f + y;
    const float corr = (y - (u - 1.0f)) * __builtin_amdgcn_rcpf(u);
    return fmaf(__builtin_amdgcn_logf(u), 0.693147180559945309f, corr);
}

// The accept statistic E + d q(y) in fp32 for a lane with 1 + c x = v0 > 0,
// and the size of its fp32 error bound (term magnitudes times a few ulp, plus
// the effect of y's own rounding): a statistic within the bound of zero is
// decided again in fp64.
struct MtStat {
    float stat, bound;
};
__device__ __forceinline__ MtStat mt_stat(float d, float y, float v0, float e) {
    const float l = log1p_fast(y);
    const float y2 = y * y;
    const float y3 = y2 * y;
    const float q = (3.0f * l - 3.0f * y) + (1.5f * y2 - y3);
    // magnitudes of the terms: 3|l| + 3|y| + 1.5 y^2 + |y|^3 (Horner in |y|)
    // and the effect of y's own rounding, 3 y^4 / v0
    const float ay = fabsf(y);
    const float poly = fmaf(ay, fmaf(ay, ay + 1.5f, 3.0f), 3.0f * fabsf(l));
    const float mag = e + d * fmaf(3.0f * y2, y2 * __builtin_amdgcn_rcpf(v0), poly);
    return MtStat{e + d * q, 2e-6f * mag};
}

// Per-lane condition from a wave mask (the mask's own lane bit, no compare).
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

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
// the source's counters).  Each round's lane conditions are wave masks: the
// ballot of one comparison is that comparison's own mask, masks combine on
// the scalar unit, and a lane reads its bit back where it needs a condition.
// Src provides:
//   float first()                 shape of this lane's first draw (any
//                                 value if it holds none)
//   bool holding()                whether this lane holds a draw (a single
//                                 comparison)
//   float complete(uint64_t md, float g, float alpha)
//                                 called by every lane with the mask of
//                                 lanes whose draw is done; such a lane hands
//                                 over g; returns the shape of the lane's
//                                 draw for the next round
//   void flush(bool final)        epoch point (global stores go here);
//                                 final at the end of the rounds
constexpr uint32_t EPOCH_ROUNDS = 4;

// COVERED: the readers' rings hold an epoch's worst case (64 Gaussians and
// 128 exponentials per round), so no call inside the rounds needs to stage.
// EPOCH (a power of two) is the number of rounds between epoch points.
// Rounds run in whole epochs: the loop stops after the first multiple of
// EPOCH rounds that is at least max_rounds, or when no lane holds a draw.
template <bool COVERED, uint32_t EPOCH = EPOCH_ROUNDS, class RN, class RE, class Src>
__device__ __forceinline__ void gamma_rounds(RN& rn, RE& re, Src& src, uint32_t max_rounds) {
    // Covered readers move only their ring positions inside an epoch.
    auto adv_n = [&](uint32_t n) {
        if constexpr (COVERED) rn.advance_pos(n); else rn.advance(n);
    };
    auto adv_e = [&](uint32_t n) {
        if constexpr (COVERED) re.advance_pos(n); else re.advance(n);
    };
    float al = src.first();
    // Let every load issued so far land here, once: otherwise the first use
    // of a loaded value inside the loop makes the compiler wait for all
    // memory operations in flight at that point of every round.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // One round for the lanes of mask mh (those holding a draw).
    auto one_round = [&](const uint64_t mh) {
        // shapes outside (0, 2^64) have no draw (it completes at once with NaN
        // and consumes nothing); below 1 the boost applies
        // from the bits: b - 1 below the bits of 2^64 less one is 0 < al <
        // 2^64 (zero, negatives and NaN wrap or lie above), below those of
        // 1 less one is 0 < al < 1
        const uint32_t b1 = __float_as_uint(al) - 1u;
        const uint64_t mv = wave_ballot(b1 < 0x5F7FFFFFu);
        const uint64_t mboost = wave_ballot(b1 < 0x3F7FFFFFu);
        // selects, not a branch: al + 1 where the boost applies, al + 0 = al
        // elsewhere (al > 0 wherever the sum is used)
        const float ab = al + (lane_in(mboost) ? 1.0f : 0.0f);
        const float a = lane_in(mv) ? ab : 1.0f;
        const float d = a - (1.0f / 3.0f);
        const float c = __builtin_amdgcn_rsqf(9.0f * d);  // 1 / sqrt(9 d)
        const uint64_t mp = mh & mv;
        // The Gaussian call and the exponential call hand entries to the
        // same lanes whenever every pending lane has 1 + c x > 0, which is
        // nearly always: both are read with the same ranks at once, and the
        // exponential call is redone with its own ranks when it is not so.
        // The rare branches are marked so, which keeps them out of line and
        // the common path free of taken branches.
        const uint32_t np = (uint32_t)__popcll(mp);
        if constexpr (!COVERED) {
            rn.reserve(np);
            re.reserve(np);
        }
        const uint32_t rk = mask_rank(mp);
        const float xr = rn.peek(rk);
        float e = re.peek(rk);
        adv_n(np);
        const float x = lane_in(mp) ? xr : 0.0f;
        const float y = c * x;
        const float v0 = 1.0f + y;
        const uint64_t me = mp & wave_ballot(v0 > 0.0f);
        if (__builtin_expect(me == mp, 1)) {
            adv_e(np);
        } else {
            e = re.peek(mask_rank(me));
            adv_e((uint32_t)__popcll(me));
        }
        // One lane in twenty-odd needs the logarithm in a round, so the wave
        // nearly always does: every lane evaluates the test, and only lanes
        // whose fp32 statistic is within its error bound of zero (rare)
        // decide again in fp64.
        const MtStat st = mt_stat(d, y, v0, e);
        uint64_t macc = me & wave_ballot(st.stat > 0.0f);
        const uint64_t muns = me & wave_ballot(!(fabsf(st.stat) > st.bound));
        if (__builtin_expect(muns != 0, 0)) {
            bool a64 = false;
            if (lane_in(muns)) a64 = mt_accept64(a, x, e);
            macc = (macc & ~muns) | (muns & wave_ballot(a64));
        }
        float g = d * (v0 * v0 * v0);
        // boost: g exp(-E'/alpha) = 2^(log2 g - E' log2(e) / alpha), one
        // exponential whose result underflows only when the product does
        const uint64_t mb = macc & mboost;
        if (mb != 0) {
            const uint32_t nb = (uint32_t)__popcll(mb);
            if constexpr (!COVERED) re.reserve(nb);
            const float e2 = re.peek(mask_rank(mb));
            adv_e(nb);
            const float gb = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(g) -
                                                    e2 * (1.44269504088896341f * __builtin_amdgcn_rcpf(al)));
            g = lane_in(mb) ? gb : g;
        }
        g = lane_in(mv) ? g : __builtin_nanf("");
        al = src.complete(mh & (macc | ~mv), g, al);
    };
    // Epochs of EPOCH rounds, the rounds of an epoch unrolled.
    bool live = true;
    for (uint32_t round = 0; live; round += EPOCH) {
        uint64_t mh = wave_ballot(src.holding());
        if (mh == 0 || round >= max_rounds) break;
        if constexpr (COVERED) {
            rn.sync_avail();
            re.sync_avail();
        }
        epoch_point(rn, re);
        src.flush();
        static_for<0, (int)EPOCH>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (!live) return;
            if (i > 0) {
                mh = wave_ballot(src.holding());
                if (__builtin_expect(mh == 0, 0)) {
                    live = false;
                    return;
                }
            }
            one_round(mh);
        });
    }
    if constexpr (COVERED) {
        rn.sync_avail();
        re.sync_avail();
    }
    src.flush(true);
}

// One draw per lane (the one-at-a-time call).
struct OneEachSrc {
    int32_t want;  // 1 while this lane's draw is pending
    float alpha;
    float g;
    __device__ __forceinline__ float first() { return want ? alpha : 1.0f; }
    __device__ __forceinline__ bool holding() const { return want != 0; }
    __device__ __forceinline__ float complete(uint64_t md, float gv, float al) {
        const bool done = lane_in(md);
        g = done ? gv : g;
        want = done ? 0 : want;
        return al;
    }
    __device__ __forceinline__ void flush(bool = false) {}
};

// Components of one Dirichlet item: lanes start with components 0..63 and a
// lane whose draw completes takes the lowest component not yet started.
// y receives component k's gamma at y[k].
struct CompSrc {
    int K;
    uint32_t next;  // wave-uniform
    int comp;
    const float* alpha;  // per component, or null: base + cnt[k]
    const int32_t* cnt;
    float* y;
    float base = 0.1f;  // prior added to the counts
    int ys = 1;         // element stride of y
    __device__ __forceinline__ float shape(int k) const {
        return alpha ? alpha[k] : base + (float)cnt[k];
    }
    __device__ __forceinline__ float first() {
        comp = (int)lane_id();
        next = (uint32_t)min(K, 64);
        return comp < K ? shape(comp) : 1.0f;
    }
    __device__ __forceinline__ bool holding() const { return comp < K; }
    __device__ __forceinline__ float complete(uint64_t md, float gv, float al) {
        const bool done = lane_in(md);
        if (done) y[(size_t)comp * ys] = gv;
        float a = al;
        if (done) {
            comp = (int)(next + mask_rank(md));
            if (comp < K) a = shape(comp);
        }
        next += (uint32_t)__popcll(md);
        return a;
    }
    __device__ __forceinline__ void flush(bool = false) {}
};

// Wave minimum / maximum of an int32 (every lane gets the result), by DPP
// lane moves: lanes without a source keep the identity.
template <bool MAX>
__device__ __forceinline__ int32_t wave_minmax(int32_t v) {
    constexpr int32_t ID = MAX ? INT32_MIN : INT32_MAX;
    auto op = [](int32_t a, int32_t b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(ID, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// The minimum of a, the maximum of b and the minimum of c over the wave, the
// three reductions interleaved step by step, so that no lane move reads a
// register written by the instruction just before it (which would need wait
// states of its own).
__device__ __forceinline__ void wave_min_max_min(int32_t a, int32_t b, int32_t c, int32_t& amin,
                                                 int32_t& bmax, int32_t& cmin) {
    auto step = [&](auto ctl) {
        constexpr int CTL = decltype(ctl)::value & 0xFFF;
        constexpr int ROWS = decltype(ctl)::value >> 12;
        a = min(a, __builtin_amdgcn_update_dpp(INT32_MAX, a, CTL, ROWS, 0xF, false));
        b = max(b, __builtin_amdgcn_update_dpp(INT32_MIN, b, CTL, ROWS, 0xF, false));
        c = min(c, __builtin_amdgcn_update_dpp(INT32_MAX, c, CTL, ROWS, 0xF, false));
    };
    step(std::integral_constant<int, 0xF111>{});  // row_shr:1
    step(std::integral_constant<int, 0xF112>{});  // row_shr:2
    step(std::integral_constant<int, 0xF114>{});  // row_shr:4
    step(std::integral_constant<int, 0xF118>{});  // row_shr:8
    step(std::integral_constant<int, 0xA142>{});  // row_bcast:15 into rows 1 and 3
    step(std::integral_constant<int, 0xC143>{});  // row_bcast:31 into rows 2 and 3
    amin = __builtin_amdgcn_readlane(a, 63);
    bmax = __builtin_amdgcn_readlane(b, 63);
    cmin = __builtin_amdgcn_readlane(c, 63);
}

// One chain per lane: g_t ~ Gamma(alpha_t, 1), alpha_{t+1} = 0.1 + g_t; the
// lane starts its next step as soon as a draw is accepted.
//
// Trace rows are staged in LDS (a ring of TRACE_ROWS rows of 64 values) and
// stored whole: a lane that completes step t writes row t of the ring, and at
// an epoch point every row below the smallest step a lane still holds is
// complete and goes out as one 256-byte row store (lanes whose chain has no
// such step, or that wrote the row in an earlier launch, are masked off).
// Lanes at different steps (rejections) then no longer scatter 4-byte stores
// over many rows.  When the lanes spread further apart than the ring holds,
// the lowest rows are stored partially (the lanes that have written them) and
// a lane that later completes such a row stores its value directly.  Where
// every lane of the wave has written four consecutive rows in this launch
// (and the trace rows are 16-byte aligned), the four rows go out in one
// 16-byte store per lane: lane l stores chains 4 (l mod 16) .. + 3 of row
// r + l / 16.
constexpr int32_t TRACE_ROWS = 16;
template <bool SUMS>
struct ChainSrc {
    int32_t t, L;
    int32_t t0;      // the lane's first step in this launch
    float alpha;
    bool trace;      // wave-uniform: write the trace
    bool vec;        // wave-uniform: trace rows 16-byte aligned (four-row stores)
    int32_t t0max;   // wave-uniform: the largest t0 of the wave
    float* col;      // this lane's trace column (row 0), or null
    int64_t stride;  // trace elements between steps
    float* ring;     // LDS, TRACE_ROWS x 64 values; this lane's column
    int32_t f;       // wave-uniform: rows below f have been stored
    double s1, s2;   // SUMS: the sum and sum of squares of this lane's
                     // draws, in step order
    __device__ __forceinline__ float first() {
        t0 = t;
        t0max = wave_minmax<true>(t0);
        // the smallest step a lane still holds; the largest step when no lane
        // holds one (a finished unit launched again), so that f stays a row
        // number and the flush's row arithmetic cannot overflow
        f = min(wave_minmax<false>(t < L ? t : INT32_MAX), t0max);
        return alpha;
    }
    __device__ __forceinline__ bool holding() const { return t < L; }
    // Every lane writes its value to the ring slot of its current step (also
    // without a trace: the ring is there either way); only lanes whose draw
    // completed move on, so a slot written by a lane that did not is
    // rewritten before its row is stored.  A lane behind the stored rows
    // stores a completed value itself; its ring write is harmless: the slot's
    // earlier row has gone out, and its next row is stored for this lane only
    // after the lane has passed it, i.e. rewritten the slot.
    __device__ __forceinline__ float complete(uint64_t md, float gv, float) {
        const bool done = lane_in(md);
        const bool behind = t < f;
        ring[(t & (TRACE_ROWS - 1)) * 64] = gv;
        if (behind && done && trace) col[(int64_t)t * stride] = gv;
        if constexpr (SUMS) {
            if (done) {
                const double d = (double)gv;
                s1 += d;
                s2 = fma(d, d, s2);  // d * d is exact: the same as a rounded product
            }
        }
        alpha = done ? 0.1f + gv : alpha;
        t += done ? 1 : 0;
        return alpha;
    }
    // Row r: the lanes that wrote it in this launch store their value.
    __device__ __forceinline__ void store_row(int32_t r) {
        if (t0 <= r && r < t) col[(int64_t)r * stride] = ring[(r & (TRACE_ROWS - 1)) * 64];
    }
    // Rows r .. r + 3, written by every lane in this launch: lane l moves
    // chains 4 (l mod 16) .. 4 (l mod 16) + 3 of row r + l / 16 (16 bytes
    // from the ring, 16 bytes to the trace).
    __device__ __forceinline__ void store_rows4(int32_t r) {
        const uint32_t lane = lane_id();
        const int32_t rr = r + (int32_t)(lane >> 4);
        const uint32_t cc = 4u * (lane & 15u);
        const float4 v = *reinterpret_cast<const float4*>(
            ring - lane + (uint32_t)(rr & (TRACE_ROWS - 1)) * 64u + cc);
        *reinterpret_cast<float4*>(col - lane + (int64_t)rr * stride + cc) = v;
    }
    // Epoch point (final: the end of the launch, when every written row goes
    // out).  Keeps room in the ring for the next EPOCH_ROUNDS steps.
    __device__ __forceinline__ void flush(bool final = false) {
        int32_t lo, hi, tmin;
        wave_min_max_min(t < L ? t : INT32_MAX, t, t, lo, hi, tmin);
        if (trace) {
            const int32_t end = final ? hi : min(lo, hi);
            // f <= hi and every bound below is at least -TRACE_ROWS, so no
            // sum or difference here overflows
            int32_t r = f;
            // every lane has written rows below the smallest t of the wave
            if (vec && r >= t0max) {
                const int32_t lim = min(end, tmin) - 3;
                for (; r < lim; r += 4) store_rows4(r);
            }
            // rows below end are complete; rows below hi + EPOCH_ROUNDS -
            // TRACE_ROWS go out partially, making room in the ring
            const int32_t nf = max(end, hi + (int32_t)EPOCH_ROUNDS - TRACE_ROWS);
            for (; r < nf; ++r) store_row(r);
            f = max(f, nf);
        } else {
            f = max(f, max(min(lo, hi), hi + (int32_t)EPOCH_ROUNDS - TRACE_ROWS));
        }
    }
};

// Inclusive prefix sums over the 64 lanes with DPP lane moves (no LDS):
// four row shifts give the sums within each row of 16 lanes, then the last
// lane of row 0 (of row 2) is added to row 1 (row 3), and the last lane of
// row 1 to rows 2 and 3.  Lanes without a source add zero.  The order of
// additions is fixed, so float sums are reproducible.
template <int CTRL, int ROWS, bool BOUND_ZERO, class T>
__device__ __forceinline__ T dpp_move(T x) {
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int32_t, x), CTRL, ROWS, 0xF, BOUND_ZERO));
}
template <class T>
__device__ __forceinline__ T dpp_incl_scan(T v) {
    v += dpp_move<0x111, 0xF, true>(v);   // row_shr:1
    v += dpp_move<0x112, 0xF, true>(v);   // row_shr:2
    v += dpp_move<0x114, 0xF, true>(v);   // row_shr:4
    v += dpp_move<0x118, 0xF, true>(v);   // row_shr:8
    v += dpp_move<0x142, 0xA, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xC, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the wave, identical in every lane (the scan's last lane).
__device__ __forceinline__ float wave_sum(float v) {
    const float t = dpp_incl_scan(v);
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, t), 63));
}

// Sum over an aligned group of S lanes (S = 8 or 16), identical in every
// lane of the group, by DPP lane moves (no LDS round trip): for S = 16 each
// lane first adds the lane 8 away in its row (a rotation by 8 within the
// row of 16), so lanes j and j + 8 hold the same pair sum; then within each
// half-row lane j adds lane 7 - j (half mirror), and the four distinct pair
// sums of a quad are added by the quad exchanges (lanes differing in bit 0,
// then bit 1).  Floating-point addition is commutative, so every lane of
// the group forms the same sum.  For a group of 16 whose upper 8 lanes hold
// zero the first step adds zero to each value, so the sum equals that of the
// lower 8 lanes as a group of 8: documents of up to 8 components get the
// same sum in either layout, and in the wave of a single document.
template <int S>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (S >= 16) v = v + dpp_move<0x128, 0xF, false>(v);  // row_ror:8
    v = v + dpp_move<0x141, 0xF, false>(v);  // row_half_mirror
    v = v + dpp_move<0xB1, 0xF, false>(v);   // quad_perm [1,0,3,2]
    v = v + dpp_move<0x4E, 0xF, false>(v);   // quad_perm [2,3,0,1]
    return v;
}

// Inclusive prefix sum over lanes (integers, exact).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) { return dpp_incl_scan(v); }

// Value of lane 63 (wave-uniform).
__device__ __forceinline__ int32_t last_lane(int32_t v) { return __builtin_amdgcn_readlane(v, 63); }

}  // namespace brng
