// Multi-request launches: one kernel over the units of several requests,
// each with its own descriptor, unit tables and pools, of one model or of
// several (the wave then picks its model's code).  The requests' slots sit
// in a device table written by small copy launches whose kernel arguments
// carry the slots (no host-to-device copy and no allocation, so the whole
// sequence can be captured in a graph and replayed).  Used by the batched
// form of brng_run_gibbs (requests sharing a context) and by the served
// form's ticks (requests with their own memory).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/brng.h"
#include "models.hpp"

namespace brng {

struct SlotDev {
    DescDev D;
    Meta* meta;         // unit tables; unit u of the request is meta[D.unit_base + u]
    Pools P;            // pools; the same indexing
    uint32_t unit_end;  // units of slots 0..this one (inclusive prefix)
    uint32_t pad;
};

// Slots per copy launch (its kernel argument stays under 4 KiB).
constexpr int PUT_CHUNK = 16;
struct SlotChunk {
    SlotDev s[PUT_CHUNK];
    uint32_t base;  // first table entry written
    uint32_t n;     // slots in use
};
static_assert(sizeof(SlotChunk) <= 4000, "kernel argument size");
static_assert(sizeof(SlotDev) % 4 == 0, "slots are copied as 32-bit words");

// Bytes of LDS one wave of `model` uses.
int model_lds_bytes_host(int model);

// Units of a request (64 chains each, or one document for LDA) and its
// device descriptor (step0 = 0).
uint32_t desc_unit_count(const brng_gibbs_desc& d);
DescDev desc_to_device(const brng_gibbs_desc& d);

// Write slots[0..n) (unit_end filled in here) to the device table `tab`
// (at least n entries) and launch one kernel over all their units on
// `stream`, with at most `wpb` waves per workgroup: the model's own kernel
// when every slot has the same model, else the kernel that dispatches per
// wave.  Returns BRNG_OK or BRNG_E_HIP.
brng_status launch_slots(SlotDev* slots, uint32_t n, SlotDev* tab, hipStream_t stream, int wpb);

}  // namespace brng
