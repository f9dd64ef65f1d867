// Pool windows in HBM and the per-wavefront buffer management.
//
// The paper's buffer management (Sec. 2.2, RNG functions; Sec. 2.4 lists its
// four costs: check the counter, fetch, increment, reset after refill) is
// done here once per wavefront instead of once per deviate:
//   - a unit (64 chains = one wave, or one item) owns one window per kind in
//     HBM, a run of W consecutive pool entries starting at `wbase`;
//   - a call hands one entry to every active lane: a ballot gives the active
//     mask, mbcnt the lane's rank among active lanes, popcount the number of
//     entries taken; the cursor lives in scalar registers;
//   - the staged reader copies the window through a small LDS ring, 1 KiB
//     per 128-bit load instruction, prefetching a few chunks ahead in
//     registers so HBM latency hides behind the chain arithmetic;
//   - when a window runs out the wave regenerates it in place (the paper's
//     blocking refill, Sec. 2.2), with the same Philox blocks a bulk fill
//     would write, so results never depend on the window length.
#pragma once
#include "philox.hpp"

namespace brng {

// Per-unit bookkeeping, one record per context unit (96 bytes).
struct Meta {
    uint64_t cur[4];    // entries consumed, per kind
    uint64_t wbase[4];  // pool index of window element 0, per kind
    uint32_t wlen[4];   // valid window entries (0 = empty), per kind
    uint32_t key_unit;  // Philox key word 0: request-local unit id
    uint32_t pad;
    uint64_t key_seed;  // stream seed
};
static_assert(sizeof(Meta) == 96, "Meta layout");

__device__ __forceinline__ Key meta_key(const Meta& m) {
    Key k;
    k.k0 = m.key_unit;
    k.k1 = (uint32_t)m.key_seed;
    k.c3 = (uint32_t)(m.key_seed >> 32);
    return k;
}

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Rank of this lane among the set lanes of mask m below it.
__device__ __forceinline__ uint32_t mask_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Wave-cooperative generation of `nblocks` blocks starting at block `b0`
// into `dst` (16 bytes per block, 64 lanes write 1 KiB per instruction).
template <uint32_t KIND>
__device__ __forceinline__ void gen_blocks_wave(uint4* dst, const Key& key, uint64_t b0,
                                                uint32_t nblocks) {
    const uint32_t lane = lane_id();
    for (uint32_t b = lane; b < nblocks; b += 64) dst[b] = gen_block<KIND>(key, b0 + b);
}

// Regenerate a window so that it holds entries [first, first + W); `first`
// is a multiple of 64 blocks.  The fences order this wave's earlier loads of
// the window before the overwrite, and the new stores before later loads by
// other lanes of the same wave (same CU, workgroup scope suffices).
template <uint32_t KIND>
__device__ __forceinline__ void refill_window(typename KindTraits<KIND>::T* win, const Key& key,
                                              uint64_t first, uint32_t W) {
    constexpr int EPB = KindTraits<KIND>::EPB;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    gen_blocks_wave<KIND>(reinterpret_cast<uint4*>(win), key, first / EPB, W / EPB);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// ---------------------------------------------------------------------------
// Direct reader: entries come straight from the HBM window (one call per
// launch in the step kernels, so staging would only add traffic).
// ---------------------------------------------------------------------------
template <uint32_t KIND>
struct DirectReader {
    using T = typename KindTraits<KIND>::T;
    static constexpr uint32_t CH = 64 * KindTraits<KIND>::EPB;  // alignment of window starts
    T* win;
    Key key;
    uint64_t wbase, cur;
    uint32_t wlen, W;

    __device__ void open(const Meta& m, T* pool_unit, uint32_t Wk) {
        win = pool_unit;
        key = meta_key(m);
        wbase = m.wbase[KIND];
        wlen = m.wlen[KIND];
        cur = m.cur[KIND];
        W = Wk;
    }
    __device__ __forceinline__ T take(bool active) {
        const uint64_t m = wave_ballot(active);
        const uint32_t n = (uint32_t)__popcll(m);
        const uint32_t r = mask_rank(m);
        if (cur < wbase || cur + n > wbase + wlen) {
            const uint64_t first = cur & ~(uint64_t)(CH - 1);
            refill_window<KIND>(win, key, first, W);
            wbase = first;
            wlen = W;
        }
        const T v = active ? win[cur + r - wbase] : T(0);
        cur += n;
        return v;
    }
    __device__ void close(Meta& m) const {
        if (lane_id() == 0) {
            m.cur[KIND] = cur;
            m.wbase[KIND] = wbase;
            m.wlen[KIND] = wlen;
        }
    }
};

// ---------------------------------------------------------------------------
// Staged reader: the window streams through an LDS ring of two chunks
// (a chunk = one 16-byte load per lane = 256 floats or 128 doubles), with
// DEPTH further chunks in flight in registers.
// ---------------------------------------------------------------------------
constexpr int STAGE_DEPTH = 3;
constexpr int RING_BYTES = 2048;  // two chunks

template <uint32_t KIND>
struct StagedReader {
    using T = typename KindTraits<KIND>::T;
    static constexpr int EPL = KindTraits<KIND>::EPB;  // entries per lane per chunk
    static constexpr uint32_t CH = 64 * EPL;
    static constexpr uint32_t R = 2 * CH;
    T* win;
    T* ring;  // LDS, R entries
    Key key;
    uint64_t wbase, cur, staged, front;
    uint32_t wlen, W;
    uint4 pf[STAGE_DEPTH];

    __device__ __forceinline__ uint4 load_chunk(uint64_t f) {
        if (f < wbase || f + CH > wbase + wlen) {
            refill_window<KIND>(win, key, f, W);
            wbase = f;
            wlen = W;
        }
        const uint4* src = reinterpret_cast<const uint4*>(win + (f - wbase));
        return src[lane_id()];
    }
    __device__ void open(const Meta& m, T* pool_unit, uint32_t Wk, T* lds_ring) {
        win = pool_unit;
        ring = lds_ring;
        key = meta_key(m);
        wbase = m.wbase[KIND];
        wlen = m.wlen[KIND];
        cur = m.cur[KIND];
        W = Wk;
        staged = cur & ~(uint64_t)(CH - 1);
        front = staged;
#pragma unroll
        for (int i = 0; i < STAGE_DEPTH; ++i) {
            pf[i] = load_chunk(front);
            front += CH;
        }
    }
    // Make entries [.., need) readable from the ring.
    __device__ __forceinline__ void ensure(uint64_t need) {
        while (staged < need) {
            uint4* dst = reinterpret_cast<uint4*>(ring + (staged & (R - 1)));
            dst[lane_id()] = pf[0];
#pragma unroll
            for (int i = 0; i + 1 < STAGE_DEPTH; ++i) pf[i] = pf[i + 1];
            pf[STAGE_DEPTH - 1] = load_chunk(front);
            front += CH;
            staged += CH;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // One call: every active lane gets the next entry, in lane order.
    __device__ __forceinline__ T take(bool active) {
        const uint64_t m = wave_ballot(active);
        const uint32_t n = (uint32_t)__popcll(m);
        const uint32_t r = mask_rank(m);
        ensure(cur + n);
        const T v = ring[(cur + r) & (R - 1)];
        cur += n;
        return active ? v : T(0);
    }
    // A call with every lane active (no ballot needed).
    __device__ __forceinline__ T take_all() {
        ensure(cur + 64);
        const T v = ring[(cur + lane_id()) & (R - 1)];
        cur += 64;
        return v;
    }
    __device__ void close(Meta& m) const {
        if (lane_id() == 0) {
            m.cur[KIND] = cur;
            m.wbase[KIND] = wbase;
            m.wlen[KIND] = wlen;
        }
    }
};

}  // namespace brng
