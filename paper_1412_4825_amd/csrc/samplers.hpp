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
// such lanes return NaN instead of looping.
__device__ __forceinline__ bool gamma_shape_ok(float alpha) {
    return alpha > 0.0f && alpha < 0x1p64f;
}

constexpr int MT_MAX_ROUNDS = 4096;  // never reached for valid shapes

// One gamma call over the lanes of a wave (active lanes draw one deviate
// each).  RN / RE are the readers of the Gaussian and exponential pools.
template <class RN, class RE>
__device__ __forceinline__ float gamma_call(RN& rn, RE& re, bool active, float alpha) {
    const bool valid = active && gamma_shape_ok(alpha);
    const bool boost = valid && alpha < 1.0f;
    const float a = valid ? (boost ? alpha + 1.0f : alpha) : 1.0f;
    const float d = a - (1.0f / 3.0f);
    const float c = 1.0f / (3.0f * sqrtf(d));
    bool pending = valid;
    float g = __builtin_nanf("");
    for (int round = 0; round < MT_MAX_ROUNDS; ++round) {
        if (wave_ballot(pending) == 0) break;
        const float x = rn.take(pending);
        const float y = c * x;
        const float v0 = 1.0f + y;
        const bool need_e = pending && v0 > 0.0f;
        const float e = re.take(need_e);
        if (need_e) {
            const float l = log1pf(y);
            const float y2 = y * y;
            const float y3 = y2 * y;
            const float q = (3.0f * l - 3.0f * y) + (1.5f * y2 - y3);
            const float stat = e + d * q;
            // bound on the fp32 evaluation error (terms' magnitudes times a
            // few ulp, plus the effect of y's own rounding)
            const float mag = e + d * (3.0f * fabsf(l) + 3.0f * fabsf(y) + 1.5f * y2 + fabsf(y3) +
                                       3.0f * y2 * y2 / v0);
            bool acc;
            if (fabsf(stat) > 1e-6f * mag)
                acc = stat > 0.0f;
            else
                acc = mt_accept64(a, x, e);
            if (acc) {
                g = d * (v0 * v0 * v0);
                pending = false;
            }
        }
    }
    const float e2 = re.take(boost);
    if (boost) g = g * expf(-e2 / alpha);
    return g;
}

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
