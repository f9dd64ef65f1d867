// Multi-request launches: one kernel of a model over the units of up to
// MULTI_MAX requests, each with its own descriptor, unit tables and pools.
// The table travels as a kernel argument (no device copy, so the launch can
// be captured in a graph and needs no allocation).  Used by the batched form
// of brng_run_gibbs (requests sharing a context) and by the served form's
// ticks (requests with their own memory).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/brng.h"
#include "models.hpp"

namespace brng {

constexpr int MULTI_MAX = 16;

struct SlotDev {
    DescDev D;
    Meta* meta;         // unit tables; unit u of the request is meta[D.unit_base + u]
    Pools P;            // pools; the same indexing
    uint32_t unit_end;  // units of slots 0..this one (inclusive prefix)
    uint32_t pad;
};

struct SlotTable {
    SlotDev s[MULTI_MAX];
    uint32_t n;            // slots in use, 1..MULTI_MAX
    uint32_t total_units;  // s[n - 1].unit_end
};
static_assert(sizeof(SlotTable) <= 4000, "kernel argument size");

// Bytes of LDS one wave of `model` uses.
int model_lds_bytes_host(int model);

// Units of a request (64 chains each, or one document for LDA) and its
// device descriptor (step0 = 0).
uint32_t desc_unit_count(const brng_gibbs_desc& d);
DescDev desc_to_device(const brng_gibbs_desc& d);

// Launch the model's multi-request kernel over T on `stream`, with at most
// `wpb` waves per workgroup.  Returns BRNG_OK or BRNG_E_HIP.
brng_status launch_slots(int model, const SlotTable& T, hipStream_t stream, int wpb);

}  // namespace brng
