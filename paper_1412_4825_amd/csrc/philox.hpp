// Core engine and base-deviate conversions, device side (gfx950).
//
// The paper keeps "buffers of random deviates for reducible distributions
// (uniform, Gaussian, exponential)" that a vector engine refills in bulk
// (Sec. 2.1, Key Concepts; Sec. 2.2, Implementation).  The engine here is
// the counter-based Philox4x32-10 generator (Salmon, Moraes, Dror & Shaw,
// SC'11): one 128-bit counter block gives four 32-bit words, so any pool
// entry is a pure function of (seed, unit, kind, index) and a window can be
// regenerated anywhere, by any wave, in any order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace brng {

enum : uint32_t { KIND_U = 0, KIND_N = 1, KIND_E = 2, KIND_U64 = 3 };

struct Key {
    uint32_t k0;     // unit id (request-local)
    uint32_t k1;     // seed, low 32 bits
    uint32_t c3;     // seed, high 32 bits (fourth counter word)
};

// Ten Philox4x32 rounds.  Each round multiplies c0 and c2 by the Philox
// constants (full 64-bit products, one v_mad_u64_u32 each), swaps the halves
// and mixes in the key; the key advances by the Weyl increments between
// rounds.  Key words are wave-uniform in every caller, so the key schedule
// runs on the scalar unit.
// KEYS_AT_USE: the bumped keys are recomputed at each use (two scalar adds
// per round) instead of being hoisted out of the caller's loops, where twenty
// loop-invariant scalar registers would crowd out a sampler's own state (the
// gamma and Dirichlet rounds); callers with few live scalars keep them.
template <bool KEYS_AT_USE = false>
__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
    if (KEYS_AT_USE) {
        k0 = __builtin_amdgcn_readfirstlane(k0);
        k1 = __builtin_amdgcn_readfirstlane(k1);
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input xor in one gfx950 instruction (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Two counters under one key schedule (the key words advance once for both):
// what a lane computes when it regenerates two blocks of one window.
template <bool KEYS_AT_USE = false>
__device__ __forceinline__ void philox10x2(uint32_t (&a)[4], uint32_t (&b)[4], uint32_t k0,
                                           uint32_t k1) {
    if (KEYS_AT_USE) {
        k0 = __builtin_amdgcn_readfirstlane(k0);
        k1 = __builtin_amdgcn_readfirstlane(k1);
        asm volatile("" : "+s"(k0), "+s"(k1));
    }
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa0 = (uint64_t)a[0] * 0xD2511F53u;
        const uint64_t pa1 = (uint64_t)a[2] * 0xCD9E8D57u;
        const uint64_t pb0 = (uint64_t)b[0] * 0xD2511F53u;
        const uint64_t pb1 = (uint64_t)b[2] * 0xCD9E8D57u;
        const uint32_t na0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa1 >> 32), a[1], k0, 0x96);
        const uint32_t na2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa0 >> 32), a[3], k1, 0x96);
        const uint32_t nb0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb1 >> 32), b[1], k0, 0x96);
        const uint32_t nb2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb0 >> 32), b[3], k1, 0x96);
        a[1] = (uint32_t)pa1;
        a[3] = (uint32_t)pa0;
        a[0] = na0;
        a[2] = na2;
        b[1] = (uint32_t)pb1;
        b[3] = (uint32_t)pb0;
        b[0] = nb0;
        b[2] = nb2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

template <bool KEYS_AT_USE = false>
__device__ __forceinline__ uint4 block_words(const Key& key, uint32_t kind, uint64_t block) {
    return philox10<KEYS_AT_USE>((uint32_t)block, (uint32_t)(block >> 32), kind, key.c3, key.k0,
                                 key.k1);
}

// U = (2 (w >> 9) + 1) 2^-24: the open midpoint grid, exact in fp32.
// Formed from the bits of 1 + (w >> 9) 2^-23 minus (1 - 2^-24): both
// operands lie in [1/2, 2) within a factor of two of each other, so the
// difference is exact (one shift, one or and one subtraction).
__device__ __forceinline__ float u01(uint32_t w) {
    return __uint_as_float((w >> 9) | 0x3F800000u) - 0x1.fffffep-1f;
}

// U64 = (2k + 1) 2^-53 with k = (wa << 20) | (wb >> 12): 52 random bits.
__device__ __forceinline__ double u01d(uint32_t wa, uint32_t wb) {
    const uint64_t k = ((uint64_t)wa << 20) | (uint64_t)(wb >> 12);
    return (double)(2 * k + 1) * 0x1p-53;
}

// E = -ln U = -ln 2 * log2 U.  U is a normal fp32 number in [2^-24, 1), so
// the hardware base-2 logarithm needs no range handling; one product with ln 2
// follows (a few ulp in all).
__device__ __forceinline__ float neg_ln(float u) {
    return __builtin_amdgcn_logf(u) * -0.693147180559945309f;
}
__device__ __forceinline__ float expo(uint32_t w) { return neg_ln(u01(w)); }

// sin and cos of 2 pi u for u on the uniform grid (u in (0,1)).  The
// reduction is exact: t = 4u and k = rint(t) are exact, f = t - k is exact
// and lies in [-1/2, 1/2], so 2 pi u = (pi/2)(k + f) and only a = (pi/2) f,
// |a| <= pi/4, goes through the Taylor polynomials (the first omitted terms
// are below 3e-9 relative).  The quadrant k mod 4 rotates the pair.
__device__ __forceinline__ float2 sincos_2pi(float u) {
    const float t = 4.0f * u;
    const float kf = rintf(t);
    const float f = t - kf;
    const float a = f * 1.57079632679489662f;
    const float a2 = a * a;
    float s = fmaf(a2, 2.75573192e-6f, -1.98412698e-4f);  // 1/9!, -1/7!
    s = fmaf(a2, s, 8.33333333e-3f);                       // 1/5!
    s = fmaf(a2, s, -1.66666667e-1f);                      // -1/3!
    s = fmaf(a2 * a, s, a);
    float c = fmaf(a2, 2.48015873e-5f, -1.38888889e-3f);  // 1/8!, -1/6!
    c = fmaf(a2, c, 4.16666667e-2f);                       // 1/4!
    c = fmaf(a2, c, -0.5f);
    c = fmaf(a2, c, 1.0f);
    const uint32_t k = (uint32_t)(int)kf;
    const float ss = (k & 1) ? c : s;  // sin(theta + k pi/2)
    const float cc = (k & 1) ? s : c;
    // the sign changes (bit 1 of k for the sine, of k + 1 for the cosine)
    // applied to the sign bit directly
    const uint32_t fs = (k << 30) & 0x80000000u;
    const uint32_t fc = ((k + 1u) << 30) & 0x80000000u;
    const float sn = __uint_as_float(__float_as_uint(ss) ^ fs);
    const float cs = __uint_as_float(__float_as_uint(cc) ^ fc);
    return make_float2(sn, cs);
}

// Box-Muller: radius from the first word, angle 2 pi Ub from the second;
// cosine goes to the even entry, sine to the odd one.
__device__ __forceinline__ float2 box_muller(uint32_t wa, uint32_t wb) {
    const float r = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(u01(wa)) * -1.38629436111989061f);
    const float2 sc = sincos_2pi(u01(wb));
    return make_float2(r * sc.y, r * sc.x);
}

// Four words -> the raw bits of their entries (four floats, or two doubles
// for U64), ready for one 128-bit store.
template <uint32_t KIND>
__device__ __forceinline__ uint4 convert_block(const uint4 w) {
    if constexpr (KIND == KIND_U) {
        return make_uint4(__float_as_uint(u01(w.x)), __float_as_uint(u01(w.y)),
                          __float_as_uint(u01(w.z)), __float_as_uint(u01(w.w)));
    } else if constexpr (KIND == KIND_E) {
        return make_uint4(__float_as_uint(expo(w.x)), __float_as_uint(expo(w.y)),
                          __float_as_uint(expo(w.z)), __float_as_uint(expo(w.w)));
    } else if constexpr (KIND == KIND_N) {
        const float2 a = box_muller(w.x, w.y);
        const float2 b = box_muller(w.z, w.w);
        return make_uint4(__float_as_uint(a.x), __float_as_uint(a.y), __float_as_uint(b.x),
                          __float_as_uint(b.y));
    } else {
        const double a = u01d(w.x, w.y);
        const double b = u01d(w.z, w.w);
        const uint64_t ia = (uint64_t)__double_as_longlong(a);
        const uint64_t ib = (uint64_t)__double_as_longlong(b);
        return make_uint4((uint32_t)ia, (uint32_t)(ia >> 32), (uint32_t)ib, (uint32_t)(ib >> 32));
    }
}

// Pool block `block` of (key, KIND), converted.
template <uint32_t KIND, bool KEYS_AT_USE = false>
__device__ __forceinline__ uint4 gen_block(const Key& key, uint64_t block) {
    return convert_block<KIND>(block_words<KEYS_AT_USE>(key, KIND, block));
}

// Pool blocks `ba` and `bb` of (key, KIND), converted, with one key schedule.
template <uint32_t KIND, bool KEYS_AT_USE = false>
__device__ __forceinline__ void gen_block2(const Key& key, uint64_t ba, uint64_t bb, uint4& va,
                                           uint4& vb) {
    uint32_t a[4] = {(uint32_t)ba, (uint32_t)(ba >> 32), KIND, key.c3};
    uint32_t b[4] = {(uint32_t)bb, (uint32_t)(bb >> 32), KIND, key.c3};
    philox10x2<KEYS_AT_USE>(a, b, key.k0, key.k1);
    va = convert_block<KIND>(make_uint4(a[0], a[1], a[2], a[3]));
    vb = convert_block<KIND>(make_uint4(b[0], b[1], b[2], b[3]));
}

template <uint32_t KIND> struct KindTraits {
    using T = float;
    static constexpr int EPB = 4;  // entries per Philox block / per 16-byte store
};
template <> struct KindTraits<KIND_U64> {
    using T = double;
    static constexpr int EPB = 2;
};

}  // namespace brng
