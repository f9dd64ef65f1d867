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
#include <type_traits>

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

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

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
    // Make entries [cur, cur + n) readable.
    __device__ __forceinline__ void reserve(uint32_t n) {
        if (cur < wbase || cur + n > wbase + wlen) {
            const uint64_t first = cur & ~(uint64_t)(CH - 1);
            refill_window<KIND>(win, key, first, W);
            wbase = first;
            wlen = W;
        }
    }
    // Entry cur + r; r up to 64 is safe after reserve (clamped to the window).
    __device__ __forceinline__ T peek(uint32_t r) const {
        const uint64_t i = cur + r;
        return win[(i < wbase + wlen ? i : wbase + wlen - 1) - wbase];
    }
    __device__ __forceinline__ void advance(uint32_t n) { cur += n; }
    __device__ __forceinline__ T take(bool active) {
        const uint64_t m = wave_ballot(active);
        const uint32_t n = (uint32_t)__popcll(m);
        reserve(n);
        const T v = active ? peek(mask_rank(m)) : T(0);
        advance(n);
        return v;
    }
    __device__ __forceinline__ bool room() const { return false; }
    __device__ __forceinline__ void put() {}
    __device__ __forceinline__ void prefetch() {}
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
// (a chunk = one 16-byte load per lane = 256 floats or 128 doubles), the
// next chunk already in flight in a register while the current one is read.
// Runs on this path (uneven lengths, rejection loops) keep several waves per
// SIMD busy, which hides the rest of the memory latency.
// ---------------------------------------------------------------------------
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
    uint4 pf;  // chunk `staged`, in flight

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
        pf = load_chunk(staged);
        front = staged + CH;
    }
    // Make entries [.., need) readable from the ring.
    __device__ __forceinline__ void ensure(uint64_t need) {
        while (staged < need) {
            reinterpret_cast<uint4*>(ring + (staged & (R - 1)))[lane_id()] = pf;
            pf = load_chunk(front);
            front += CH;
            staged += CH;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ void reserve(uint32_t n) { ensure(cur + n); }
    __device__ __forceinline__ T peek(uint32_t r) const { return ring[((uint32_t)cur + r) & (R - 1)]; }
    __device__ __forceinline__ void advance(uint32_t n) { cur += n; }
    // One call: every active lane gets the next entry, in lane order.
    __device__ __forceinline__ T take(bool active) {
        const uint64_t m = wave_ballot(active);
        const uint32_t n = (uint32_t)__popcll(m);
        reserve(n);
        const T v = peek(mask_rank(m));
        advance(n);
        return active ? v : T(0);
    }
    __device__ __forceinline__ bool room() const { return false; }
    __device__ __forceinline__ void put() {}
    __device__ __forceinline__ void prefetch() {}
    __device__ void close(Meta& m) const {
        if (lane_id() == 0) {
            m.cur[KIND] = cur;
            m.wbase[KIND] = wbase;
            m.wlen[KIND] = wlen;
        }
    }
};

// Compile-time loop: f(integral_constant<int, J>) for J = I .. N-1.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Native four-word vector (kept in registers where HIP's uint4 struct is not).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Epoch reader: the staged reader for rejection loops, where the number of
// entries a call takes is only known at the call.  On gfx9 one counter
// tracks every outstanding vector memory operation, loads and stores alike,
// so waiting for a prefetched chunk also waits for whatever was issued after
// it.  The caller therefore stages all its readers together at fixed points
// ("epochs", every few rounds of its loop) and issues its own global stores
// right after them: each wait then covers only operations issued one epoch
// earlier.  A chunk is CHV 16-byte blocks per lane (CH entries); the LDS ring
// holds two chunks and the next chunk waits in registers.  A chunk inside
// the unit's window (the bulk fill's, in HBM) is loaded from it one epoch
// ahead; a chunk past the window is the buffer's refill, and the wave
// generates it in registers when it is staged: the entries are the same
// pure function of their index that a regenerated window would hold, and
// nothing is written back (a window written to HBM only to be read back
// once cost a quarter of the LDA kernel's time, the stores holding up the
// next loads on the shared counter).  If a call needs more than the ring
// holds, it stages at once (correct, only slower); sized so that an epoch's
// worst case fits, that never happens.
// ---------------------------------------------------------------------------
// PAIRED: a lane computes its blocks two at a time under one key schedule
// (fewer scalar instructions, more code and registers; it pays off for a
// kernel with two readers, not with three); with one block per lane per
// chunk the second block is the next chunk's, which then waits in registers.
// MIRROR: the ring is followed by a copy of its first 64 entries, so that the
// 64 entries from any position are contiguous; without it a read wraps its
// index (one more instruction) and the ring takes 256 bytes less LDS.
// WINDOW: chunks inside the pool's window are loaded from it.  Without it
// every chunk is generated (the same entries the window holds), so the
// staging registers never wait for a load: on gfx9 one counter tracks loads
// and stores alike, and a wait for a load that may be in flight also waits
// for every store the wave has issued (a chain's trace rows).
template <uint32_t KIND, int CHV, bool PAIRED = false, bool MIRROR = true, bool WINDOW = true>
struct EpochReader {
    static_assert(CHV == 1 || CHV == 2, "a chunk is one or two blocks per lane");
    using T = typename KindTraits<KIND>::T;
    static constexpr int EPB = KindTraits<KIND>::EPB;
    static constexpr uint32_t CH = 64u * EPB * CHV;
    static constexpr uint32_t R = 2 * CH;
    static constexpr int LDS_BYTES = (int)((R + (MIRROR ? 64 : 0)) * sizeof(T));
    T* win;
    T* ring;  // LDS, R entries (+ 64: the mirror)
    Key key;
    uint64_t wbase, staged;  // ring holds entries [.., staged)
    uint32_t wlen, W;
    int32_t avail;  // staged - cursor (the cursor itself is staged - avail)
    uint32_t pos;   // cursor mod R: the ring index of the next entry
    bool inflight;  // pf holds chunk `staged`
    bool ahead;     // pf holds chunk `staged`, generated with the previous one
    u32x4 pf[CHV];

    __device__ __forceinline__ bool in_window(uint64_t f) const {
        return f >= wbase && f + CH <= wbase + wlen;
    }
    __device__ __forceinline__ void load(uint64_t f) {
        const u32x4* src = reinterpret_cast<const u32x4*>(win + (f - wbase)) + lane_id();
#pragma unroll
        for (int j = 0; j < CHV; ++j) pf[j] = src[j * 64];
    }
    // Whether the ring has room for the waiting chunk.
    __device__ __forceinline__ bool room() const { return avail <= (int32_t)(R - CH); }
    // Move chunk `staged` into the ring (needs room()).  Without a waiting
    // copy the chunk is generated here.
    __device__ __forceinline__ void put() {
        const uint32_t off = (uint32_t)staged & (R - 1);
        u32x4* dst = reinterpret_cast<u32x4*>(ring + off) + lane_id();
        u32x4 head;
        if (inflight) {
#pragma unroll
            for (int j = 0; j < CHV; ++j) dst[j * 64] = pf[j];
            head = pf[0];
        } else {
            const uint32_t lane = lane_id();
            const uint64_t b0 = staged / EPB;
            u32x4 tmp[CHV];
            if constexpr (PAIRED) {
                uint4 va, vb;
                gen_block2<KIND, true>(key, b0 + lane, b0 + 64 + lane, va, vb);
                tmp[0] = u32x4{va.x, va.y, va.z, va.w};
                if constexpr (CHV == 2) {
                    tmp[1] = u32x4{vb.x, vb.y, vb.z, vb.w};
                } else {
                    pf[0] = u32x4{vb.x, vb.y, vb.z, vb.w};  // the next chunk
                    ahead = true;
                }
            } else {
#pragma unroll
                for (int j = 0; j < CHV; ++j) {
                    const uint4 v = gen_block<KIND, true>(key, b0 + (uint32_t)(j * 64) + lane);
                    tmp[j] = u32x4{v.x, v.y, v.z, v.w};
                }
            }
#pragma unroll
            for (int j = 0; j < CHV; ++j) dst[j * 64] = tmp[j];
            head = tmp[0];
        }
        // the mirror: entries 0..63 of the ring are lanes 0 .. 64/EPB - 1 of
        // the first load of the chunk at offset 0
        if (MIRROR && off == 0 && lane_id() < 64u / EPB)
            reinterpret_cast<u32x4*>(ring + R)[lane_id()] = head;
        staged += CH;
        avail += (int32_t)CH;
    }
    // Prefetch chunk `staged` when it lies inside the window (or keep the
    // one generated ahead).
    __device__ __forceinline__ void prefetch() {
        if (ahead) {
            ahead = false;
            inflight = true;
            return;
        }
        inflight = WINDOW && in_window(staged);
        if (inflight) load(staged);
    }
    __device__ __forceinline__ void stage() {
        put();
        prefetch();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ __forceinline__ void open(const Meta& m, T* pool_unit, uint32_t Wk, T* lds_ring) {
        win = pool_unit;
        ring = lds_ring;
        key = meta_key(m);
        wbase = m.wbase[KIND];
        wlen = m.wlen[KIND];
        W = Wk;
        const uint64_t cur = m.cur[KIND];
        staged = cur & ~(uint64_t)(CH - 1);
        avail = -(int32_t)(cur - staged);
        pos = (uint32_t)cur & (R - 1);
        ahead = false;
        prefetch();
        stage();
    }
    // Make entries [cursor, cursor + n) readable (n <= 64).
    __device__ __forceinline__ void reserve(uint32_t n) {
        while ((int32_t)n > avail) stage();
    }
    // Entry cursor + r (r < 64, after reserve).
    __device__ __forceinline__ T peek(uint32_t r) const {
        return MIRROR ? ring[pos + r] : ring[(pos + r) & (R - 1)];
    }
    __device__ __forceinline__ void advance(uint32_t n) {
        pos = (pos + n) & (R - 1);
        avail -= (int32_t)n;
    }
    // Covered use: calls move only the ring position, and the count of
    // entries left is recovered from it where it is needed (epoch points,
    // close).  Valid while 1 <= avail <= R, which holds at every epoch point
    // when an epoch never takes more than one chunk.
    __device__ __forceinline__ void advance_pos(uint32_t n) { pos = (pos + n) & (R - 1); }
    __device__ __forceinline__ void sync_avail() {
        avail = (int32_t)((((uint32_t)staged - pos - 1u) & (R - 1)) + 1u);
    }
    // One call: every active lane gets the next entry, in lane order.
    __device__ __forceinline__ T take(bool active) {
        const uint64_t m = wave_ballot(active);
        const uint32_t n = (uint32_t)__popcll(m);
        reserve(n);
        const T v = peek(mask_rank(m));
        advance(n);
        return active ? v : T(0);
    }
    __device__ void close(Meta& m) const {
        if (lane_id() == 0) {
            m.cur[KIND] = staged - (uint64_t)(int64_t)avail;
            m.wbase[KIND] = wbase;
            m.wlen[KIND] = wlen;
        }
    }
};

// Epoch point for a set of readers: every ring with room takes its waiting
// chunk, and only then are the next chunks requested, so that no reader's
// wait (for its own, epoch-old prefetch) also waits for a load just issued.
template <class... Rs>
__device__ __forceinline__ void epoch_point(Rs&... rs) {
    const bool go[] = {rs.room()...};
    int i = 0;
    ((go[i++] ? rs.put() : void()), ...);
    i = 0;
    ((go[i++] ? rs.prefetch() : void()), ...);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Lane pipe: the reader for runs where all 64 lanes take one entry per call
// for a known number of calls.  A "block" consumes one chunk's worth of
// entries (CH / 64 calls).  Chunks are loaded PIPE_DEPTH blocks ahead into
// registers that the caller indexes statically (the block loop is unrolled by
// PIPE_DEPTH with static_for), so every load has PIPE_DEPTH blocks of work
// to hide behind and no register is ever indexed at run time.  The window is
// checked once per PIPE_DEPTH blocks (cover), so the unrolled body holds no
// branch with stores in it and the compiler can count outstanding loads.
// The LDS ring holds four chunks; a block reads from two of them.
// ---------------------------------------------------------------------------
constexpr int PIPE_DEPTH = 8;
constexpr int PIPE_RING_BYTES = 4096;

template <uint32_t KIND>
struct LanePipe {
    using T = typename KindTraits<KIND>::T;
    static constexpr int EPL = KindTraits<KIND>::EPB;
    static constexpr uint32_t CH = 64 * EPL;
    static constexpr uint32_t R = 4 * CH;
    // smallest window the pipe can work with: PIPE_DEPTH + 1 chunks
    static constexpr uint32_t MIN_WINDOW = (PIPE_DEPTH + 1) * CH;
    T* win;
    T* ring;
    Key key;
    uint64_t wbase, pos, next, last;
    uint32_t wlen, W;
    uint4 pf[PIPE_DEPTH];

    // Make the window hold chunks [c, c_end] (c_end - c < W / CH).
    __device__ __forceinline__ void cover(uint64_t c, uint64_t c_end) {
        const uint64_t f = c * CH, g = (c_end + 1) * CH;
        if (f < wbase || g > wbase + wlen) {
            refill_window<KIND>(win, key, f, W);
            wbase = f;
            wlen = W;
        }
    }
    __device__ __forceinline__ uint4 raw_load(uint64_t c) const {
        return reinterpret_cast<const uint4*>(win + (c * CH - wbase))[lane_id()];
    }
    __device__ __forceinline__ void put(uint64_t c, const uint4& v) {
        reinterpret_cast<uint4*>(ring + ((c * CH) & (R - 1)))[lane_id()] = v;
    }
    // Prepare for `calls` calls of 64 entries each (calls >= 1).
    __device__ void open(const Meta& m, T* pool_unit, uint32_t Wk, T* lds_ring, uint32_t calls) {
        win = pool_unit;
        ring = lds_ring;
        key = meta_key(m);
        wbase = m.wbase[KIND];
        wlen = m.wlen[KIND];
        W = Wk;
        pos = m.cur[KIND];
        const uint64_t c0 = pos / CH;
        last = (pos + 64ull * calls - 1) / CH;
        cover(c0, min(last, c0 + PIPE_DEPTH));
        put(c0, raw_load(c0));
        next = c0 + 1;
        static_for<0, PIPE_DEPTH>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if (next + j <= last) pf[j] = raw_load(next + j);
        });
    }
    // Before blocks sb .. sb + PIPE_DEPTH - 1: the window must hold the
    // chunks they will prefetch.
    __device__ __forceinline__ void prepare(uint64_t sb) {
        const uint64_t c = next + sb + PIPE_DEPTH;
        if (c <= last) cover(c, min(last, c + PIPE_DEPTH - 1));
    }
    // Before block b (J = b % PIPE_DEPTH): stage chunk next + b from register
    // slot J and load chunk next + b + PIPE_DEPTH into it.
    template <int J>
    __device__ __forceinline__ void advance(uint64_t b) {
        const uint64_t c = next + b;
        if (c <= last) put(c, pf[J]);
        if (c + PIPE_DEPTH <= last) pf[J] = raw_load(c + PIPE_DEPTH);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // advance() for a block known to be inside the run with its prefetch
    // inside it too: no conditions at all.
    template <int J>
    __device__ __forceinline__ void advance_fast(uint64_t b) {
        const uint64_t c = next + b;
        put(c, pf[J]);
        pf[J] = raw_load(c + PIPE_DEPTH);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // Number of leading blocks for which advance_fast is valid.
    __device__ __forceinline__ uint64_t fast_blocks() const {
        return (last >= next + PIPE_DEPTH) ? last - next - PIPE_DEPTH + 1 : 0;
    }
    // Entry of call i of the current block for this lane.
    __device__ __forceinline__ T get(int i) const {
        return ring[(pos + 64u * (uint32_t)i + lane_id()) & (R - 1)];
    }
    __device__ __forceinline__ void consume(uint32_t calls) { pos += 64ull * calls; }
    __device__ void close(Meta& m) const {
        if (lane_id() == 0) {
            m.cur[KIND] = pos;
            m.wbase[KIND] = wbase;
            m.wlen[KIND] = wlen;
        }
    }
};

}  // namespace brng
