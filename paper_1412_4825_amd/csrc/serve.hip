// Served form: a request loop with continuous batching (host side).
//
// The paper keeps its buffers inside one sampler object and refills them
// when they run out, and names an asynchronous refill service as future work
// (Sec. 3).  Here every admitted request owns unit tables and pools carved
// out of one device arena (admission by footprint), stays resident between
// ticks, and advances by a time slice per tick; all admitted requests share
// one multi-request launch per tick (each wave runs its request's model).
// Requests are independent (their streams are keyed by their own
// seed and request-local unit ids), and a time slice is a resume of the
// same kernel, so a served request's results equal a plain run's.
//
// Ticks complete in stream order; each tick records an event, and the host
// retires a tick once the event has passed.  At most two ticks are in flight,
// so requests that arrive meanwhile join at the next tick.  Models whose
// steps are one round each (triangle, normal/exponential, exponential, LDA
// sweeps) are sliced by steps, and the host knows when they finish.  Gamma
// chains are sliced by rounds of the rejection loop (slicing by steps would
// change which lanes share a round, hence the values); each slot's step count
// stays on the device and each unit reports in host-visible memory when its
// chains are done, which the host reads when the tick retires.  A request's
// memory is freed when the last tick that includes it has retired.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/brng.h"
#include "slots.hpp"

using namespace brng;

namespace {

constexpr uint64_t ARENA_ALIGN = 256;

uint64_t round_up(uint64_t x) { return (x + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1); }

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator over the arena's byte range; free blocks coalesce.
struct Arena {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    void init(uint64_t bytes) {
        free_.clear();
        free_[0] = bytes;
    }
    bool alloc(uint64_t size, uint64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size) continue;
            *off = it->first;
            const uint64_t rest = it->second - size, o = it->first + size;
            free_.erase(it);
            if (rest) free_[o] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t size) {
        auto it = free_.emplace(off, size).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Pool kinds a model reads.
void model_kinds(int model, bool need[4]) {
    for (int k = 0; k < 4; ++k) need[k] = false;
    switch (model) {
        case BRNG_MODEL_TRIANGLE_F64: need[BRNG_U64] = true; break;
        case BRNG_MODEL_NORMEXP:
        case BRNG_MODEL_GAMMA_CHAIN: need[BRNG_N] = need[BRNG_E] = true; break;
        case BRNG_MODEL_EXP_CHAIN: need[BRNG_E] = true; break;
        default: need[BRNG_U] = need[BRNG_N] = need[BRNG_E] = true; break;
    }
}

size_t kind_bytes(int k) { return k == BRNG_U64 ? sizeof(double) : sizeof(float); }

// Element sizes of the two traces of a model (0: none).
void trace_elems(int model, size_t* e1, size_t* e2) {
    switch (model) {
        case BRNG_MODEL_TRIANGLE_F64: *e1 = *e2 = sizeof(double); break;
        case BRNG_MODEL_NORMEXP: *e1 = *e2 = sizeof(float); break;
        case BRNG_MODEL_LDA: *e1 = sizeof(float); *e2 = sizeof(int32_t); break;
        default: *e1 = sizeof(float); *e2 = 0; break;
    }
}

struct Req {
    uint64_t ticket;
    brng_gibbs_desc d;
    uint64_t t_arrive, t_admit, t_done;
    uint64_t off, bytes;
    uint64_t status_off;   // gamma: unit_done bytes in the host-visible buffer
    uint32_t n_units;
    int32_t done;          // steps launched (step-sliced models)
    uint64_t last_tick;    // newest tick that includes it
    uint64_t final_tick;   // step-sliced: the tick that completes it
    bool finished;         // completion seen
    Meta* meta;
    Pools P;
    int32_t* progress;     // gamma: steps done per slot
    uint8_t* unit_done;    // gamma: per unit, 1 when its chains are done
};

struct Tick {
    uint64_t id;
    hipEvent_t ev;
    std::vector<Req*> reqs;
};

bool round_sliced(int model) { return model == BRNG_MODEL_GAMMA_CHAIN; }

}  // namespace

struct brng_server {
    brng_serve_config cfg;
    hipStream_t stream;
    char* base;
    Arena arena;
    SlotDev* table;   // slots of one tick (max_active entries)
    uint8_t* status;  // host-visible unit_done bytes of gamma requests
    Arena status_arena;
    uint64_t in_use, peak;
    std::deque<Req*> waiting;
    std::vector<Req*> active;
    std::deque<Tick> ticks;
    std::vector<hipEvent_t> spare;
    std::deque<brng_serve_done> done;
    uint64_t next_ticket, n_ticks, n_completed;
};

namespace {

uint64_t footprint(const brng_server* s, const brng_gibbs_desc& d) {
    const uint64_t nu = desc_unit_count(d);
    bool need[4];
    model_kinds(d.model, need);
    uint64_t b = round_up(nu * sizeof(Meta));
    for (int k = 0; k < 4; ++k)
        if (need[k]) b += round_up(nu * (uint64_t)s->cfg.window[k] * kind_bytes(k));
    if (round_sliced(d.model)) b += round_up(nu * 64 * sizeof(int32_t));
    return b;
}

// Carve the request's unit tables and pools out of its arena block.
void carve(brng_server* s, Req* r) {
    char* p = s->base + r->off;
    r->meta = reinterpret_cast<Meta*>(p);
    p += round_up((uint64_t)r->n_units * sizeof(Meta));
    bool need[4];
    model_kinds(r->d.model, need);
    void* pool[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int k = 0; k < 4; ++k) {
        if (!need[k]) continue;
        pool[k] = p;
        p += round_up((uint64_t)r->n_units * s->cfg.window[k] * kind_bytes(k));
    }
    r->P.u = (float*)pool[BRNG_U];
    r->P.n = (float*)pool[BRNG_N];
    r->P.e = (float*)pool[BRNG_E];
    r->P.u64 = (double*)pool[BRNG_U64];
    for (int k = 0; k < 4; ++k) r->P.W[k] = need[k] ? s->cfg.window[k] : 0;
    r->progress = round_sliced(r->d.model) ? reinterpret_cast<int32_t*>(p) : nullptr;
}

brng_status get_event(brng_server* s, hipEvent_t* ev) {
    if (!s->spare.empty()) {
        *ev = s->spare.back();
        s->spare.pop_back();
        return BRNG_OK;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess ? BRNG_OK : BRNG_E_HIP;
}

void release(brng_server* s, Req* r, brng_status st) {
    brng_serve_done o;
    o.ticket = r->ticket;
    o.t_arrive_ns = r->t_arrive;
    o.t_admit_ns = r->t_admit;
    o.t_done_ns = r->t_done;
    o.status = st;
    o.pad = 0;
    s->done.push_back(o);
    s->arena.release(r->off, r->bytes);
    if (r->unit_done) s->status_arena.release(r->status_off, r->n_units);
    s->in_use -= r->bytes;
    ++s->n_completed;
    delete r;
}

void drop_active(brng_server* s, Req* r) {
    auto it = std::find(s->active.begin(), s->active.end(), r);
    if (it != s->active.end()) s->active.erase(it);
}

// Retire ticks whose event has passed (in order).
brng_status retire(brng_server* s) {
    while (!s->ticks.empty()) {
        Tick& t = s->ticks.front();
        const hipError_t q = hipEventQuery(t.ev);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return BRNG_E_HIP;
        const uint64_t now = now_ns();
        for (Req* r : t.reqs) {
            if (!r->finished) {
                bool fin;
                if (round_sliced(r->d.model)) {
                    fin = true;
                    for (uint32_t u = 0; u < r->n_units && fin; ++u) fin = r->unit_done[u] != 0;
                    if (fin) drop_active(s, r);
                } else {
                    fin = r->final_tick == t.id;
                }
                if (fin) {
                    r->finished = true;
                    r->t_done = now;
                }
            }
            if (r->finished && r->last_tick == t.id) release(s, r, BRNG_OK);
        }
        s->spare.push_back(t.ev);
        s->ticks.pop_front();
    }
    return BRNG_OK;
}

// Place r in the arena (and its status bytes); false when it does not fit.
bool place(brng_server* s, Req* r) {
    uint64_t off, soff = 0;
    if (!s->arena.alloc(r->bytes, &off)) return false;
    if (round_sliced(r->d.model) && !s->status_arena.alloc(r->n_units, &soff)) {
        s->arena.release(off, r->bytes);
        return false;
    }
    r->off = off;
    carve(s, r);
    if (r->progress) {
        r->status_off = soff;
        r->unit_done = s->status + soff;
        std::memset(r->unit_done, 0, r->n_units);
        (void)hipMemsetAsync(r->progress, 0, (size_t)r->n_units * 64 * sizeof(int32_t),
                             s->stream);
    }
    r->t_admit = now_ns();
    s->in_use += r->bytes;
    s->peak = std::max(s->peak, s->in_use);
    s->active.push_back(r);
    return true;
}

// Admission by footprint, in submission order, except that while the oldest
// waiting request does not fit, later ones that fit are admitted past it
// (looking at most SCAN_AHEAD requests ahead) until it has waited
// max_bypass_ms since its arrival; after that nothing passes it, so memory
// freed by finishing requests goes to it and it cannot starve.
constexpr int SCAN_AHEAD = 64;

void admit(brng_server* s) {
    const uint64_t bypass_ns = (uint64_t)s->cfg.max_bypass_ms * 1000000ull;
    const uint64_t now = now_ns();
    int scanned = 0;
    auto it = s->waiting.begin();
    while (it != s->waiting.end() && s->active.size() < s->cfg.max_active &&
           scanned < SCAN_AHEAD) {
        Req* r = *it;
        if (place(s, r)) {
            it = s->waiting.erase(it);
            continue;
        }
        if (it == s->waiting.begin()) {
            const bool aged = now >= r->t_arrive && now - r->t_arrive >= bypass_ns;
            if (bypass_ns == 0 || aged) break;  // the head waits; nothing passes it
        }
        ++it;
        ++scanned;
    }
}

// One tick: every admitted request advances by its model's slice, all in one
// launch.
brng_status launch_tick(brng_server* s) {
    Tick t;
    t.id = s->n_ticks + 1;
    brng_status st = get_event(s, &t.ev);
    if (st != BRNG_OK) return st;
    std::vector<SlotDev> slots;
    slots.reserve(s->active.size());
    std::vector<Req*> still;
    still.reserve(s->active.size());
    for (Req* r : s->active) {
        const int m = r->d.model;
        DescDev D = desc_to_device(r->d);
        D.unit_base = 0;
        D.flags = r->last_tick ? FLAG_RESUME : 0u;
        bool last = false;
        if (round_sliced(m)) {
            D.max_rounds = (int32_t)s->cfg.tick_steps;
            D.progress = r->progress;
            D.unit_done = r->unit_done;
        } else {
            const int32_t slice =
                (int32_t)(m == BRNG_MODEL_LDA ? s->cfg.tick_sweeps : s->cfg.tick_steps);
            const int32_t steps = std::min(slice, r->d.max_steps - r->done);
            D.max_steps = steps;
            D.step0 = r->done;
            size_t e1, e2;
            trace_elems(m, &e1, &e2);
            const int64_t row = (int64_t)r->done * r->d.trace_stride;
            if (D.trace) D.trace = (char*)D.trace + row * (int64_t)e1;
            if (D.trace2 && e2) D.trace2 = (char*)D.trace2 + row * (int64_t)e2;
            r->done += steps;
            last = r->done >= r->d.max_steps;
        }
        SlotDev S;
        std::memset(&S, 0, sizeof(S));
        S.D = D;
        S.meta = r->meta;
        S.P = r->P;
        slots.push_back(S);
        r->last_tick = t.id;
        t.reqs.push_back(r);
        if (last)
            r->final_tick = t.id;
        else
            still.push_back(r);
    }
    st = launch_slots(slots.data(), (uint32_t)slots.size(), s->table, s->stream, 4);
    if (st != BRNG_OK) return st;
    if (hipEventRecord(t.ev, s->stream) != hipSuccess) return BRNG_E_HIP;
    s->active.swap(still);
    s->ticks.push_back(std::move(t));
    ++s->n_ticks;
    return BRNG_OK;
}

brng_status check_request(const brng_server* s, const brng_gibbs_desc& d) {
    if (d.model < 0 || d.model >= BRNG_NMODELS) return BRNG_E_ARG;
    if (d.n_chains == 0 || d.max_steps < 0 || !d.d_state) return BRNG_E_ARG;
    if (d.unit_base != 0 || d.flags != 0) return BRNG_E_ARG;
    const int64_t width = d.model == BRNG_MODEL_LDA ? 0 : (int64_t)d.n_chains;
    if ((d.d_trace || d.d_trace2) && d.trace_stride < width) return BRNG_E_ARG;
    if (d.model == BRNG_MODEL_LDA && (!d.d_offsets || !d.d_ntok)) return BRNG_E_ARG;
    bool need[4];
    model_kinds(d.model, need);
    for (int k = 0; k < 4; ++k)
        if (need[k] && !s->cfg.window[k]) return BRNG_E_KIND_DISABLED;
    return BRNG_OK;
}

bool window_ok(uint32_t W) {
    return W == 0 || (W % BRNG_WINDOW_ALIGN == 0 && W >= BRNG_WINDOW_MIN);
}

}  // namespace

extern "C" {

uint64_t brng_serve_now(void) { return now_ns(); }

brng_status brng_serve_open(const brng_serve_config* cfg, brng_server** out) {
    if (!out) return BRNG_E_ARG;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget == 0 || cfg->max_active == 0 || cfg->tick_steps == 0 ||
        cfg->tick_sweeps == 0)
        return BRNG_E_ARG;
    for (int k = 0; k < 4; ++k)
        if (!window_ok(cfg->window[k])) return BRNG_E_ARG;
    brng_server* s = new (std::nothrow) brng_server();
    if (!s) return BRNG_E_NOMEM;
    s->cfg = *cfg;
    s->stream = (hipStream_t)cfg->hip_stream;
    s->base = nullptr;
    const uint64_t bytes = round_up(cfg->hbm_budget);
    if (hipMalloc((void**)&s->base, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return BRNG_E_NOMEM;
    }
    s->arena.init(bytes);
    s->table = nullptr;
    if (hipMalloc((void**)&s->table, sizeof(SlotDev) * cfg->max_active) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(s->base);
        delete s;
        return BRNG_E_NOMEM;
    }
    // unit_done bytes: a gamma unit's footprint is well above 2 KiB
    const uint64_t sbytes = bytes / 2048 + 4096;
    s->status = nullptr;
    if (hipHostMalloc((void**)&s->status, sbytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(s->table);
        (void)hipFree(s->base);
        delete s;
        return BRNG_E_NOMEM;
    }
    s->status_arena.init(sbytes);
    s->in_use = s->peak = 0;
    s->next_ticket = 1;
    s->n_ticks = s->n_completed = 0;
    *out = s;
    return BRNG_OK;
}

brng_status brng_serve_submit(brng_server* s, const brng_gibbs_desc* d, uint64_t t_arrive_ns,
                              uint64_t* ticket) {
    if (!s || !d || !ticket) return BRNG_E_ARG;
    const brng_status st = check_request(s, *d);
    if (st != BRNG_OK) return st;
    const uint64_t fp = footprint(s, *d);
    if (fp > round_up(s->cfg.hbm_budget)) return BRNG_E_NOMEM;
    Req* r = new (std::nothrow) Req();
    if (!r) return BRNG_E_NOMEM;
    r->ticket = s->next_ticket++;
    r->d = *d;
    r->t_arrive = t_arrive_ns ? t_arrive_ns : now_ns();
    r->t_admit = 0;
    r->off = 0;
    r->bytes = fp;
    r->t_done = 0;
    r->status_off = 0;
    r->n_units = desc_unit_count(*d);
    r->done = 0;
    r->last_tick = r->final_tick = 0;
    r->finished = false;
    r->meta = nullptr;
    r->progress = nullptr;
    r->unit_done = nullptr;
    s->waiting.push_back(r);
    *ticket = r->ticket;
    return BRNG_OK;
}

brng_status brng_serve_progress(brng_server* s, int32_t wait) {
    if (!s) return BRNG_E_ARG;
    const size_t before = s->ticks.size();
    brng_status st = retire(s);
    if (st != BRNG_OK) return st;
    if (wait && !s->ticks.empty() && s->ticks.size() == before) {
        if (hipEventSynchronize(s->ticks.front().ev) != hipSuccess) return BRNG_E_HIP;
        st = retire(s);
        if (st != BRNG_OK) return st;
    }
    admit(s);
    if (!s->active.empty() && s->ticks.size() < 2) return launch_tick(s);
    return BRNG_OK;
}

brng_status brng_serve_poll(brng_server* s, brng_serve_done* out, uint32_t cap, uint32_t* n) {
    if (!s || !n || (cap && !out)) return BRNG_E_ARG;
    uint32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return BRNG_OK;
}

brng_status brng_serve_stats_get(const brng_server* s, brng_serve_stats* o) {
    if (!s || !o) return BRNG_E_ARG;
    o->waiting = (uint32_t)s->waiting.size();
    o->active = (uint32_t)s->active.size();
    o->ticks_in_flight = (uint32_t)s->ticks.size();
    o->pad = 0;
    o->bytes_in_use = s->in_use;
    o->bytes_peak = s->peak;
    o->ticks = s->n_ticks;
    o->completed = s->n_completed;
    return BRNG_OK;
}

brng_status brng_serve_close(brng_server* s) {
    if (!s) return BRNG_OK;
    brng_status st = BRNG_OK;
    while (st == BRNG_OK && (!s->waiting.empty() || !s->active.empty() || !s->ticks.empty()))
        st = brng_serve_progress(s, 1);
    if (st != BRNG_OK) {
        // a failed launch: drain the stream and drop what is left
        (void)hipStreamSynchronize(s->stream);
        for (Tick& t : s->ticks) s->spare.push_back(t.ev);
    }
    std::vector<Req*> left(s->waiting.begin(), s->waiting.end());
    left.insert(left.end(), s->active.begin(), s->active.end());
    for (Tick& t : s->ticks) left.insert(left.end(), t.reqs.begin(), t.reqs.end());
    std::sort(left.begin(), left.end());
    left.erase(std::unique(left.begin(), left.end()), left.end());
    for (Req* r : left) delete r;
    for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
    (void)hipHostFree(s->status);
    (void)hipFree(s->table);
    (void)hipFree(s->base);
    delete s;
    return st;
}

}  // extern "C"
