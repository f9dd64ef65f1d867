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
    int32_t step0;  // steps already taken (time-sliced runs): per-chain
                    // lengths count from here; traces start at row 0
    // Round-sliced gamma chains (the served form): steps done per slot,
    // rounds to run (0: until every chain is done) and, per unit, 1 once all
    // its chains are done (host-visible memory); null/0 in plain runs.
    int32_t max_rounds;
    int32_t* progress;
    uint8_t* unit_done;
    // Per-chain (LDA: per-component) sums of each output and of its square
    // over this launch's steps, added to what the array holds, or null:
    // [output][2][chains or components], fp64, one add per output per step
    // in step order (so a run sliced over several launches gives the same
    // sums as one launch).
    double* sums;
};

enum : int32_t { M_TRIANGLE = 0, M_NORMEXP = 1, M_GAMMA = 2, M_LDA = 3, M_EXPCHAIN = 4 };
enum : uint32_t { FLAG_RESUME = 1u };

// LDA's per-wave auxiliary LDS area: bin boundaries, counts and component
// gammas (256 each).
constexpr int AUX_BYTES = 3072;

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

// q + x * x with the product rounded before the sum (never one fused
// multiply-add), as the sums of squares are defined.
__device__ __forceinline__ double add_square(double q, double x) {
#pragma clang fp contract(off)
    return q + x * x;
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
    const int32_t L = in ? (D.steps ? D.steps[chain] - D.step0 : D.max_steps) : 0;
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
    const size_t n = D.n_chains;
    double sx = 0.0, sxx = 0.0, sy = 0.0, syy = 0.0;
    if (D.sums && in) {
        sx = D.sums[chain];
        sxx = D.sums[n + chain];
        sy = D.sums[2 * n + chain];
        syy = D.sums[3 * n + chain];
    }
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
            if (D.sums) {
                sx += x;
                sxx = add_square(sxx, x);
                sy += y;
                syy = add_square(syy, y);
            }
        }
    }
    if (in) {
        st[chain] = x;
        st[(size_t)D.n_chains + chain] = y;
        if (D.sums) {
            D.sums[chain] = sx;
            D.sums[n + chain] = sxx;
            D.sums[2 * n + chain] = sy;
            D.sums[3 * n + chain] = syy;
        }
    }
    ru.close(*mp);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Output staging for the full-occupancy paths: four steps of one output go
// through LDS so that each lane stores 16 bytes (four consecutive chains of
// one step) instead of 4 bytes per step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool aligned16(const void* p, int64_t stride) {
    return ((uintptr_t)p & 15) == 0 && (stride & 3) == 0;
}

// ob: 256 floats of LDS holding [step i][lane] for the block's four steps.
__device__ __forceinline__ void store4(float* ob, float* trace, int64_t stride, uint32_t slot0,
                                       uint32_t t0) {
    const uint32_t lane = lane_id();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float4 v = reinterpret_cast<const float4*>(ob)[lane];
    float* dst = trace + (size_t)(t0 + (lane >> 4)) * stride + slot0 + 4 * (lane & 15);
    *reinterpret_cast<float4*>(dst) = v;
}

// Running sum and sum of squares of one fp32 output in fp64: v and v * v are
// exact in fp64, so each step rounds once per sum.
struct Sum2 {
    double s = 0.0, q = 0.0;
    __device__ __forceinline__ void add(float v) {
        const double d = (double)v;
        s += d;
        q = add_square(q, d);
    }
    __device__ __forceinline__ void load(const double* p, size_t n, size_t i) {
        s = p[i];
        q = p[n + i];
    }
    __device__ __forceinline__ void store(double* p, size_t n, size_t i) const {
        p[i] = s;
        p[n + i] = q;
    }
};

// ---------------------------------------------------------------------------
// Normal/exponential chain: s' = 0.9 s + (0.5 + |s|) z, e = E / (1 + s'^2).
// Fresh chains draw s_0 as their first Gaussian.
// ---------------------------------------------------------------------------
constexpr int NORMEXP_LDS_BYTES = 2 * PIPE_RING_BYTES + 2048;

__device__ void unit_normexp(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                             unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot0 = local * 64;
    const uint32_t slot = slot0 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;  // a bad permutation entry idles the lane
    const int32_t L = in ? (D.steps ? D.steps[chain] - D.step0 : D.max_steps) : 0;
    const bool fresh = !(D.flags & FLAG_RESUME);
    Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    float* pool_n = P.n + (size_t)gu * P.W[KIND_N];
    float* pool_e = P.e + (size_t)gu * P.W[KIND_E];
    float* st = reinterpret_cast<float*>(D.state);
    float* ts = reinterpret_cast<float*>(D.trace);
    float* te = reinterpret_cast<float*>(D.trace2);
    const int32_t smax = D.max_steps;
    // the pipelined path serves runs without sums; sums take the staged one
    const bool full = smax > 0 && !D.sums && P.W[KIND_N] >= LanePipe<KIND_N>::MIN_WINDOW &&
                      P.W[KIND_E] >= LanePipe<KIND_E>::MIN_WINDOW &&
                      (wave_ballot(in && L >= smax) == ~0ull);
    const size_t n = D.n_chains;
    Sum2 ss, se;  // sums of s' and e (outputs 0 and 1)
    if (D.sums && in) {
        ss.load(D.sums, n, chain);
        se.load(D.sums + 2 * n, n, chain);
    }
    float s;
    if (full) {
        if (fresh) {  // s_0: one call on the Gaussian pool
            DirectReader<KIND_N> r0;
            r0.open(m, pool_n, P.W[KIND_N]);
            s = r0.take(true);
            m.cur[KIND_N] = r0.cur;
            m.wbase[KIND_N] = r0.wbase;
            m.wlen[KIND_N] = r0.wlen;
        } else {
            s = st[chain];
        }
        LanePipe<KIND_N> pn;
        LanePipe<KIND_E> pe;
        pn.open(m, pool_n, P.W[KIND_N], reinterpret_cast<float*>(lds), (uint32_t)smax);
        pe.open(m, pool_e, P.W[KIND_E], reinterpret_cast<float*>(lds + PIPE_RING_BYTES),
                (uint32_t)smax);
        float* ob = reinterpret_cast<float*>(lds + 2 * PIPE_RING_BYTES);
        const bool vec = ts && te && aligned16(ts, D.stride) && aligned16(te, D.stride);
        const uint32_t blocks = ((uint32_t)smax + 3) / 4;
        const uint32_t nfast =
            (uint32_t)min((uint64_t)((uint32_t)smax / 4), min(pn.fast_blocks(), pe.fast_blocks()));
        // one block: 4 steps (fewer in the last block)
        auto block = [&](auto jc, uint32_t b, auto fastc, auto vecc) {
            constexpr int j = decltype(jc)::value;
            constexpr bool FAST = decltype(fastc)::value;
            constexpr bool VEC = decltype(vecc)::value;
            if constexpr (FAST) {
                pn.template advance_fast<j>(b);
                pe.template advance_fast<j>(b);
            } else {
                pn.template advance<j>(b);
                pe.template advance<j>(b);
            }
            const uint32_t t0 = 4 * b;
            const uint32_t nc = FAST ? 4u : min(4u, (uint32_t)smax - t0);
            float sp[4], ev[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (FAST || (uint32_t)i < nc) {
                    const float z = pn.get(i);
                    const float e = pe.get(i);
                    sp[i] = fmaf(0.5f + fabsf(s), z, 0.9f * s);
                    ev[i] = e / fmaf(sp[i], sp[i], 1.0f);
                    s = sp[i];
                }
            }
            if constexpr (FAST && VEC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    ob[64 * i + lane] = sp[i];
                    ob[256 + 64 * i + lane] = ev[i];
                }
                store4(ob, ts, D.stride, slot0, t0);
                store4(ob + 256, te, D.stride, slot0, t0);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (FAST || (uint32_t)i < nc) {
                        if (ts) ts[(size_t)(t0 + i) * D.stride + slot] = sp[i];
                        if (te) te[(size_t)(t0 + i) * D.stride + slot] = ev[i];
                    }
                }
            }
            pn.consume(nc);
            pe.consume(nc);
        };
        auto run = [&](auto vecc) {
            uint32_t sb = 0;
            for (; sb + PIPE_DEPTH <= nfast; sb += PIPE_DEPTH) {  // branch-free body
                pn.prepare(sb);
                pe.prepare(sb);
                static_for<0, PIPE_DEPTH>([&](auto jc) {
                    block(jc, sb + decltype(jc)::value, std::true_type{}, vecc);
                });
            }
            for (; sb < blocks; sb += PIPE_DEPTH) {  // the last few blocks
                pn.prepare(sb);
                pe.prepare(sb);
                static_for<0, PIPE_DEPTH>([&](auto jc) {
                    const uint32_t b = sb + decltype(jc)::value;
                    if (b < blocks) block(jc, b, std::false_type{}, vecc);
                });
            }
        };
        if (vec)
            run(std::true_type{});
        else
            run(std::false_type{});
        st[chain] = s;
        pn.close(*mp);
        pe.close(*mp);
    } else {
        StagedReader<KIND_N> rn;
        StagedReader<KIND_E> re;
        rn.open(m, pool_n, P.W[KIND_N], reinterpret_cast<float*>(lds));
        re.open(m, pool_e, P.W[KIND_E], reinterpret_cast<float*>(lds + RING_BYTES));
        if (fresh)
            s = rn.take(in);
        else
            s = in ? st[chain] : 0.0f;
        for (int32_t t = 0; t < smax; ++t) {
            const bool act = in && t < L;
            if (wave_ballot(act) == 0) break;
            const float z = rn.take(act);
            const float sp = fmaf(0.5f + fabsf(s), z, 0.9f * s);
            const float e = re.take(act);
            if (act) {
                const float ev = e / fmaf(sp, sp, 1.0f);
                if (ts) ts[(size_t)t * D.stride + slot] = sp;
                if (te) te[(size_t)t * D.stride + slot] = ev;
                if (D.sums) {
                    ss.add(sp);
                    se.add(ev);
                }
                s = sp;
            }
        }
        if (in) st[chain] = s;
        rn.close(*mp);
        re.close(*mp);
    }
    if (D.sums && in) {
        ss.store(D.sums, n, chain);
        se.store(D.sums + 2 * n, n, chain);
    }
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Exponential chain (served form's exponential kind): e' = E / (1 + e^2).
// Fresh chains draw e_0 as their first exponential.
// ---------------------------------------------------------------------------
constexpr int EXPCHAIN_LDS_BYTES = PIPE_RING_BYTES + 1024;

__device__ void unit_expchain(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                              unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot0 = local * 64;
    const uint32_t slot = slot0 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;
    const int32_t L = in ? (D.steps ? D.steps[chain] - D.step0 : D.max_steps) : 0;
    const bool fresh = !(D.flags & FLAG_RESUME);
    Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    float* pool_e = P.e + (size_t)gu * P.W[KIND_E];
    float* st = reinterpret_cast<float*>(D.state);
    float* tr = reinterpret_cast<float*>(D.trace);
    const int32_t smax = D.max_steps;
    const bool full = smax > 0 && !D.sums && P.W[KIND_E] >= LanePipe<KIND_E>::MIN_WINDOW &&
                      (wave_ballot(in && L >= smax) == ~0ull);
    const size_t n = D.n_chains;
    Sum2 sv;  // sums of e'
    if (D.sums && in) sv.load(D.sums, n, chain);
    float v;
    if (full) {
        if (fresh) {
            DirectReader<KIND_E> r0;
            r0.open(m, pool_e, P.W[KIND_E]);
            v = r0.take(true);
            m.cur[KIND_E] = r0.cur;
            m.wbase[KIND_E] = r0.wbase;
            m.wlen[KIND_E] = r0.wlen;
        } else {
            v = st[chain];
        }
        LanePipe<KIND_E> pe;
        pe.open(m, pool_e, P.W[KIND_E], reinterpret_cast<float*>(lds), (uint32_t)smax);
        float* ob = reinterpret_cast<float*>(lds + PIPE_RING_BYTES);
        const bool vec = tr && aligned16(tr, D.stride);
        const uint32_t blocks = ((uint32_t)smax + 3) / 4;
        const uint32_t nfast = (uint32_t)min((uint64_t)((uint32_t)smax / 4), pe.fast_blocks());
        auto block = [&](auto jc, uint32_t b, auto fastc, auto vecc) {
            constexpr int j = decltype(jc)::value;
            constexpr bool FAST = decltype(fastc)::value;
            constexpr bool VEC = decltype(vecc)::value;
            if constexpr (FAST)
                pe.template advance_fast<j>(b);
            else
                pe.template advance<j>(b);
            const uint32_t t0 = 4 * b;
            const uint32_t nc = FAST ? 4u : min(4u, (uint32_t)smax - t0);
            float ev[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (FAST || (uint32_t)i < nc) {
                    v = pe.get(i) / fmaf(v, v, 1.0f);
                    ev[i] = v;
                }
            }
            if constexpr (FAST && VEC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) ob[64 * i + lane] = ev[i];
                store4(ob, tr, D.stride, slot0, t0);
            } else {
                if (tr) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (FAST || (uint32_t)i < nc) tr[(size_t)(t0 + i) * D.stride + slot] = ev[i];
                }
            }
            pe.consume(nc);
        };
        auto run = [&](auto vecc) {
            uint32_t sb = 0;
            for (; sb + PIPE_DEPTH <= nfast; sb += PIPE_DEPTH) {
                pe.prepare(sb);
                static_for<0, PIPE_DEPTH>([&](auto jc) {
                    block(jc, sb + decltype(jc)::value, std::true_type{}, vecc);
                });
            }
            for (; sb < blocks; sb += PIPE_DEPTH) {
                pe.prepare(sb);
                static_for<0, PIPE_DEPTH>([&](auto jc) {
                    const uint32_t b = sb + decltype(jc)::value;
                    if (b < blocks) block(jc, b, std::false_type{}, vecc);
                });
            }
        };
        if (vec)
            run(std::true_type{});
        else
            run(std::false_type{});
        st[chain] = v;
        pe.close(*mp);
    } else {
        StagedReader<KIND_E> re;
        re.open(m, pool_e, P.W[KIND_E], reinterpret_cast<float*>(lds));
        if (fresh)
            v = re.take(in);
        else
            v = in ? st[chain] : 0.0f;
        for (int32_t t = 0; t < smax; ++t) {
            const bool act = in && t < L;
            if (wave_ballot(act) == 0) break;
            const float e = re.take(act);
            if (act) {
                v = e / fmaf(v, v, 1.0f);
                if (tr) tr[(size_t)t * D.stride + slot] = v;
                if (D.sums) sv.add(v);
            }
        }
        if (in) st[chain] = v;
        re.close(*mp);
    }
    if (D.sums && in) sv.store(D.sums, n, chain);
    store_key(mp, m);
}

// ---------------------------------------------------------------------------
// Varying-shape gamma chain: g_t ~ Gamma(alpha_t, 1), alpha_{t+1} = 0.1 + g_t.
// Each lane runs its chain through the gamma rounds and starts its next step
// as soon as a draw is accepted.
// ---------------------------------------------------------------------------
// Without the mirrors a wave's LDS is 10 KiB, so four workgroups of four
// waves fit a CU's 160 KiB (four waves per SIMD instead of three).  The
// readers generate every chunk, also inside the windows: the loop then holds
// no load, and its epoch points never wait for the trace stores in flight.
using GammaRN = EpochReader<KIND_N, 1, true, false, false>;
using GammaRE = EpochReader<KIND_E, 2, true, false, false>;
constexpr int GAMMA_OBUF_BYTES = TRACE_ROWS * 64 * 4;
constexpr int GAMMA_LDS_BYTES = GammaRN::LDS_BYTES + GammaRE::LDS_BYTES + GAMMA_OBUF_BYTES;
// An epoch's worst case fits the rings (a round takes at most one Gaussian
// and two exponentials per lane), so the rounds run without staging checks.
static_assert(GammaRN::CH >= 64 * EPOCH_ROUNDS && GammaRE::CH >= 128 * EPOCH_ROUNDS,
              "gamma rings must cover an epoch");

template <bool SUMS>
__device__ void unit_gamma(const DescDev& D, Meta* mp, const Pools& P, uint32_t local,
                           unsigned char* lds) {
    const uint32_t lane = lane_id();
    const uint32_t slot = local * 64 + lane;
    const bool in0 = slot < D.n_chains;
    const uint32_t chain = in0 ? (D.perm ? (uint32_t)D.perm[slot] : slot) : 0;
    const bool in = in0 && chain < D.n_chains;
    const int32_t L = in ? min(D.steps ? D.steps[chain] - D.step0 : D.max_steps, D.max_steps) : 0;
    const Meta m = open_meta(D, mp, local);
    const uint32_t gu = D.unit_base + local;
    GammaRN rn;
    GammaRE re;
    rn.open(m, P.n + (size_t)gu * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + GammaRN::LDS_BYTES));
    float* st = reinterpret_cast<float*>(D.state);
    ChainSrc<SUMS> src;
    // steps already done by this slot (round-sliced runs continue a chain
    // mid-way; the round sequence is the same as in one straight run)
    const int32_t t0 = (D.progress && in) ? D.progress[slot] : 0;
    src.t = t0;
    src.L = L;
    src.alpha = in ? st[chain] : 1.0f;
    src.trace = D.trace != nullptr;
    src.col = src.trace ? reinterpret_cast<float*>(D.trace) + slot : nullptr;
    src.stride = D.stride;
    src.vec = src.trace && ((uintptr_t)D.trace & 15u) == 0 && (D.stride & 3) == 0;
    src.ring = reinterpret_cast<float*>(lds + GammaRN::LDS_BYTES + GammaRE::LDS_BYTES) + lane;
    src.s1 = src.s2 = 0.0;
    if (SUMS && in) {
        src.s1 = D.sums[chain];
        src.s2 = D.sums[(size_t)D.n_chains + chain];
    }
    const uint32_t smax = (uint32_t)min(D.max_steps, 1 << 24);
    // Waves of longer chains issue first: they decide when the launch ends,
    // and the waves of shorter chains on the same SIMD take the slots they
    // leave.  Priority = the quarter of max_steps the wave's longest chain
    // reaches (the wave's own issue priority; results do not depend on it).
    {
        const int32_t lmax = wave_minmax<true>(L - t0);
        const int64_t pr = 4ll * lmax / ((int64_t)max(D.max_steps, 1) + 1);
        if (pr >= 3)
            __builtin_amdgcn_s_setprio(3);
        else if (pr == 2)
            __builtin_amdgcn_s_setprio(2);
        else if (pr == 1)
            __builtin_amdgcn_s_setprio(1);
    }
    gamma_rounds<true>(rn, re, src, D.max_rounds > 0 ? (uint32_t)D.max_rounds : 4096u + 64u * smax);
    if (in) st[chain] = src.alpha;
    if (SUMS && in) {
        D.sums[chain] = src.s1;
        D.sums[(size_t)D.n_chains + chain] = src.s2;
    }
    if (D.progress && in) D.progress[slot] = src.t;
    if (D.unit_done) {
        const bool all = wave_ballot(src.holding()) == 0;
        if (lane == 0) D.unit_done[local] = all ? 1 : 0;
    }
    rn.close(*mp);
    re.close(*mp);
    store_key(mp, m);
}

constexpr int LDA_KMAX = 256;
// The readers generate every chunk (no loads from the windows), so the
// epoch points never wait for the theta and count rows in flight.
using LdaRN = EpochReader<KIND_N, 1, false, true, false>;
using LdaRE = EpochReader<KIND_E, 1, false, true, false>;
constexpr int LDA_RINGS_BYTES = LdaRN::LDS_BYTES + LdaRE::LDS_BYTES;
// Epoch points every two rounds keep the one-chunk rings covered.
constexpr uint32_t LDA_EPOCH = 2;
static_assert(LdaRN::CH >= 64 * LDA_EPOCH && LdaRE::CH >= 128 * LDA_EPOCH,
              "LDA rings must cover an epoch");
constexpr int LDA_LDS_BYTES = LDA_RINGS_BYTES + AUX_BYTES;

// ---------------------------------------------------------------------------
// LDA-style document: per sweep, theta ~ Dirichlet(0.1 + counts), then
// counts ~ Multinomial(n, theta) by the integer-exact rule:
//   q_k = rint(theta_k 2^24), Q = sum q_k (all q_k = 1 when Q = 0),
//   C_k = q_0 + ... + q_k; token i takes u_i from the U pool,
//   j = (u_i 2^24 - 1) / 2, t = (j Q) >> 23, bin = first k with t < C_k.
// LDS holds the bin ends, the counts and the component gammas (K <= 256).
// Whether this lane's component of block b (components 64 b .. 64 b + 63)
// exists.  K passes through an empty asm so the comparison is made where it
// is used instead of being kept, one lane mask per block, across the sweep.
__device__ __forceinline__ bool comp_in(int K, int b, uint32_t lane) {
    int Kx = __builtin_amdgcn_readfirstlane(K);
    asm volatile("" : "+s"(Kx));
    return b * 64 + (int)lane < Kx;
}

// ---------------------------------------------------------------------------
__device__ void unit_lda(const DescDev& D, Meta* mp, const Pools& P, uint32_t doc,
                         unsigned char* lds) {
    const uint32_t lane = lane_id();
    const Meta m = open_meta(D, mp, doc);
    const uint32_t gu = D.unit_base + doc;
    const int32_t off = D.offsets[doc];
    const int K = D.offsets[doc + 1] - off;
    const int ntok = D.ntok[doc];
    // first step of the bin search, kstep = 2^kexp: the largest power of
    // two <= K - 1 (the answer is at most K - 1, and the steps add up to at
    // least that); kexp = -1 for K = 1, which needs no step
    const int kexp = K > 1 ? 31 - (int)__builtin_clz((uint32_t)(K - 1)) : -1;
    LdaRN rn;
    LdaRE re;

    rn.open(m, P.n + (size_t)gu * P.W[KIND_N], P.W[KIND_N], reinterpret_cast<float*>(lds));
    re.open(m, P.e + (size_t)gu * P.W[KIND_E], P.W[KIND_E],
            reinterpret_cast<float*>(lds + LdaRN::LDS_BYTES));
    uint64_t ucur = m.cur[KIND_U];  // the U stream's cursor (entries come from registers)
    int32_t* Cs = reinterpret_cast<int32_t*>(lds + LDA_RINGS_BYTES);  // 256 bin ends
    int32_t* cnt = Cs + LDA_KMAX;                                      // 256 counts
    float* yv = reinterpret_cast<float*>(cnt + LDA_KMAX);              // 256 gammas
    int32_t* counts = reinterpret_cast<int32_t*>(D.state) + off;
    const bool want_th = D.trace != nullptr, want_ct = D.trace2 != nullptr;
    // this lane's trace entries (component lane + 64 b of the document) of
    // the current sweep's rows; one row further per sweep
    float* thp = want_th ? reinterpret_cast<float*>(D.trace) + off + lane : nullptr;
    int32_t* ctp = want_ct ? reinterpret_cast<int32_t*>(D.trace2) + off + lane : nullptr;
    // bin ends past the last component hold a value above every token's
    // t (t < Q <= 2^24 + K), so a probe there never passes and the search
    // needs no clamp
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int k = b * 64 + (int)lane;
        if (comp_in(K, b, lane)) cnt[k] = counts[k];
        else Cs[k] = 0x7fffffff;
    }
    // sums of theta and theta^2 per component: [2][total components]
    const size_t tot = D.sums ? (size_t)D.offsets[D.n_units] : 0;
    double* sp = D.sums ? D.sums + off + lane : nullptr;
    double s1[4] = {0.0, 0.0, 0.0, 0.0}, s2[4] = {0.0, 0.0, 0.0, 0.0};
    if (sp) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (comp_in(K, b, lane)) {
                s1[b] = sp[b * 64];
                s2[b] = sp[tot + b * 64];
            }
    }
    for (int32_t sw = 0; sw < D.max_steps; ++sw) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        CompSrc src;
        src.K = K;
        src.alpha = nullptr;
        src.cnt = cnt;
        src.y = yv;
        gamma_rounds<true, LDA_EPOCH>(rn, re, src, 4096u + 64u * (uint32_t)K);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float y[4];
        float part = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            const bool in = b * 64 < K && comp_in(K, b, lane);
            y[b] = in ? yv[k] : 0.0f;
            if (in) part += y[b];
        }
        // documents of up to 16 components (all in lanes 0..15) sum in the
        // same order as when several share a wave (group_sum)
        const float S = K <= 16 ? __builtin_bit_cast(float, __builtin_amdgcn_readlane(
                                      __builtin_bit_cast(int32_t, group_sum<16>(y[0])), 0))
                                : wave_sum(part);
        // theta (each gamma times the correctly rounded 1 / S), quantised
        // weights and their prefix sums
        const float inv = 1.0f / S;
        int32_t carry = 0;
        float th[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (b * 64 < K) {
                const bool in = comp_in(K, b, lane);
                th[b] = (in && S > 0.0f) ? y[b] * inv : 0.0f;
                const int32_t q = in ? (int32_t)rintf(th[b] * 16777216.0f) : 0;
                const int32_t inc = wave_incl_scan(q) + carry;
                if (in) Cs[k] = inc;
                carry = last_lane(inc);
            } else {
                th[b] = 0.0f;
            }
        }
        int32_t Q = carry;
        if (Q == 0) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int k = b * 64 + (int)lane;
                if (b * 64 < K && comp_in(K, b, lane)) Cs[k] = k + 1;
            }
            Q = K;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (b * 64 < K && comp_in(K, b, lane)) cnt[k] = 0;
        }
        if (sp) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double t = (double)th[b];
                s1[b] += t;
                s2[b] = add_square(s2[b], t);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // The sweep's uniforms are the document's entries [cu, cu + ntok) of
        // its U stream; lane l generates Philox blocks blo + l, blo + l + 64,
        // ... in registers (the buffer's refill; the bulk-filled window is
        // not read) and bins each block's four entries that fall in the
        // range.  Entry u = (2 (w >> 9) + 1) 2^-24 gives j = (u 2^24 - 1) / 2
        // = w >> 9 and t = (j Q) >> 23; its bin is the number of k with
        // C_k <= t (the C_k do not decrease and C_{K-1} = Q > t), found by
        // binary lifting over the power-of-two steps 2^e, e = kexp .. 0, the
        // same count of steps in every lane.  The steps are unrolled from the
        // largest possible one (2^7; K <= 256) and those above kstep skipped
        // as a wave, so each probe is an LDS read at a fixed offset from the
        // position reached (at most 2 kstep - 2 <= 254); a lane's four
        // searches are independent, so their LDS reads overlap.
        {
            const uint64_t cu = ucur;
            const uint64_t blo = cu / 4, bhi = (cu + (uint32_t)max(ntok, 0) + 3) / 4;
            const uint32_t c0 = (uint32_t)cu & 3u;  // cu - 4 blo
            const uint32_t nt = (uint32_t)max(ntok, 0);
            const Key ku = meta_key(m);
            for (uint64_t r0 = blo; r0 < bhi; r0 += 64) {
                const uint64_t b = r0 + lane;
                const uint32_t bi = (uint32_t)(r0 - blo) + lane;  // b - blo
                const uint4 w = block_words<true>(ku, KIND_U, b);
                const uint32_t wv[4] = {w.x, w.y, w.z, w.w};
                int32_t* p[4] = {Cs, Cs, Cs, Cs};  // bin end of the position reached
                uint32_t t[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) t[i] = (uint32_t)(((uint64_t)(wv[i] >> 9) * (uint32_t)Q) >> 23);
                static_for<0, 8>([&](auto jc) {
                    constexpr int e = 7 - decltype(jc)::value;
                    if (e <= kexp) {
                        // the four probes first, then the four steps
                        int32_t v[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) v[i] = p[i][(1 << e) - 1];
#pragma unroll
                        for (int i = 0; i < 4; ++i) p[i] += (uint32_t)v[i] <= t[i] ? (1 << e) : 0;
                    }
                });
                // the counts sit LDA_KMAX entries past the bin ends
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // entry 4 b + i is token tk of the sweep; entries before
                    // the cursor wrap to large values
                    const uint32_t tk = 4u * bi + (uint32_t)i - c0;
                    if (tk < nt) atomicAdd(p[i] + LDA_KMAX, 1);
                }
            }
            ucur = cu + (uint32_t)max(ntok, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int k = b * 64 + (int)lane;
            if (b * 64 < K && comp_in(K, b, lane)) {
                if (want_th) thp[b * 64] = th[b];
                if (want_ct) ctp[b * 64] = cnt[k];
            }
        }
        thp += D.stride;
        ctp += D.stride;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int k = b * 64 + (int)lane;
        if (b * 64 < K && comp_in(K, b, lane)) {
            counts[k] = cnt[k];
            if (sp) {
                sp[b * 64] = s1[b];
                sp[tot + b * 64] = s2[b];
            }
        }
    }
    rn.close(*mp);
    re.close(*mp);
    if (lane == 0) {  // the U window record stays as it was opened
        mp->cur[KIND_U] = ucur;
        mp->wbase[KIND_U] = m.wbase[KIND_U];
        mp->wlen[KIND_U] = m.wlen[KIND_U];
    }
    store_key(mp, m);
}

}  // namespace brng
