/*
 * brng.h: C interface of the MI355X (gfx950) varying-parameter random number
 * library built on the buffering idea of Mahani & Sharabiani, "Efficient SIMD
 * RNG for Varying-Parameter Streams: C++ Class BatchRNG" (arXiv 1412.4825).
 *
 * The method (Sec. 2.1, Key Concepts): keep pools of standard uniform,
 * Gaussian and exponential deviates that a vector engine fills in bulk, and
 * serve samplers whose parameters change at every call (the one-at-a-time
 * scenario of Sec. 1) from those pools through a cheap transform.  Here the
 * engine is Philox4x32-10 on the GPU, a pool "unit" is 64 consecutive chains
 * (one gfx950 wavefront) or one item (a Dirichlet vector / document), and
 * thousands of chains consume their unit's pools in parallel.
 *
 * Stream contract (fixed; results never depend on window length, launch
 * shape, graph capture or tuning):
 *   Philox key = (unit id, seed low 32), counter = (block low 32,
 *   block high 32, kind, seed high 32).  Entry j of kind U/N/E is word j%4 of
 *   block j/4 (N: Box-Muller on words (0,1) and (2,3), cosine on the even
 *   entry); entry j of U64 uses words 2(j%2), 2(j%2)+1 of block j/2.
 *   U = (2(w>>9)+1) 2^-24, U64 = (2k+1) 2^-53 with k = (wa<<20)|(wb>>12),
 *   E = -ln U, N = sqrt(-2 ln Ua) cos/sin(2 pi Ub).
 *   A call gives one entry of a kind to every active slot of a unit, in
 *   ascending slot order; the unit's cursor for that kind counts entries
 *   consumed (the paper's buffer_counter, Sec. 2.2).
 *
 * Conventions for every function:
 *   - Return value: brng_status, 0 on success.  Argument errors are
 *     reported synchronously and launch nothing.  BRNG_E_HIP reports a HIP
 *     runtime failure; brng_last_hip_error() gives its hipError_t code.
 *   - Pointers named d_* are device pointers owned by the caller; they must
 *     stay valid until the context's stream has passed the call.  Pointers
 *     named h_* are host pointers.  Context-owned memory (pools, cursors)
 *     is allocated by brng_create and freed by brng_destroy only.
 *   - All device work is asynchronous on the context's stream (default
 *     stream when NULL).  A context is not thread safe; distinct contexts
 *     are independent.
 *   - Arrays are contiguous.  Precision: see brng_config.prec.
 */
#ifndef BRNG_H
#define BRNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t brng_status;
enum {
    BRNG_OK = 0,
    BRNG_E_ARG = 1,           /* invalid argument (null, size, range) */
    BRNG_E_NOMEM = 2,         /* device allocation failed */
    BRNG_E_HIP = 3,           /* HIP runtime error */
    BRNG_E_KIND_DISABLED = 4, /* call needs a pool whose window length is 0 */
    BRNG_E_BUSY = 5,          /* served form: no slot or memory available */
    BRNG_E_UNSUPPORTED = 6,   /* combination not provided (e.g. fp64 gamma) */
    BRNG_E_TOO_LARGE = 7      /* request exceeds the static scratch area */
};

/* Pool kinds (Sec. 2.1: reducible base distributions). */
enum { BRNG_U = 0, BRNG_N = 1, BRNG_E = 2, BRNG_U64 = 3, BRNG_NKINDS = 4 };
/* Precision of step-call parameter and output arrays. */
enum { BRNG_F32 = 0, BRNG_F64 = 1 };
/* What a pool unit is: 64 consecutive chains, or one item. */
enum { BRNG_LAYOUT_CHAINS = 0, BRNG_LAYOUT_ITEMS = 1 };

#define BRNG_UNIT_WIDTH 64      /* chains per unit (one wavefront) */
#define BRNG_WINDOW_ALIGN 256   /* window lengths are multiples of this */
#define BRNG_WINDOW_MIN 512     /* smallest non-zero window */

typedef struct {
    uint64_t seed;
    uint32_t n_chains;   /* chains (LAYOUT_CHAINS) or items (LAYOUT_ITEMS) */
    uint32_t layout;     /* BRNG_LAYOUT_* */
    uint32_t window[4];  /* pool window per unit per kind, in entries: 0
                            disables the kind (Sec. 2.4 zero-length buffers),
                            else a multiple of 256, at least 512 */
    int32_t prec;        /* BRNG_F32 or BRNG_F64 (F64: uniform steps only,
                            from the U64 pool) */
    void *hip_stream;    /* hipStream_t, or NULL for the default stream */
} brng_config;

typedef struct brng_ctx brng_ctx;

/* Constructor (Sec. 2.2): allocate one window per unit per enabled kind,
 * set every cursor to 0 and fill every window with its first entries.
 * Units are ceil(n_chains/64) (chains) or n_chains (items).  Unit u's
 * stream is keyed by (u, seed).  Errors: BRNG_E_ARG, BRNG_E_NOMEM,
 * BRNG_E_HIP; *out is NULL on error. */
brng_status brng_create(const brng_config *cfg, brng_ctx **out);

/* Destructor (Sec. 2.2): wait for the stream, free everything.  NULL is a
 * no-op. */
brng_status brng_destroy(brng_ctx *ctx);

/* Bulk refill (the paper's batch call of the core engine, Sec. 1 and 2.2):
 * regenerate every unit's window of `kind` starting at its cursor rounded
 * down to 256 (128 for U64) entries, with coalesced 128-bit stores.
 * Errors: BRNG_E_ARG (kind), BRNG_E_KIND_DISABLED, BRNG_E_HIP. */
brng_status brng_fill_base(brng_ctx *ctx, int32_t kind);

/* One-at-a-time calls (Sec. 1; reducible transforms of Sec. 2.1): one draw
 * per chain, parameters per chain.  Layout CHAINS.  Windows that run out
 * are refilled inside the kernel.  Arrays hold n_chains elements of the
 * context precision.
 *   uniform: out = a + (b - a) u      (U pool; U64 pool when prec = F64)
 *   normal : out = mu + sigma z       (N pool; sigma is a standard deviation)
 *   exp    : out = E / lambda         (E pool; lambda is the rate)
 *   gamma  : out ~ Gamma(alpha, 1)    (Marsaglia-Tsang on N and E pools,
 *                                      alpha < 1 boosted by exp(-E'/alpha);
 *                                      alpha > 0 required, F32 only)
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
brng_status brng_step_uniform(brng_ctx *ctx, const void *d_a, const void *d_b, void *d_out);
brng_status brng_step_normal(brng_ctx *ctx, const void *d_mu, const void *d_sigma, void *d_out);
brng_status brng_step_exp(brng_ctx *ctx, const void *d_lambda, void *d_out);
brng_status brng_step_gamma(brng_ctx *ctx, const float *d_alpha, float *d_out);

/* The paper's other irreducible samplers (Sec. 2.2: GetLaplace, GetWeibull),
 * one draw per chain from the exponential pool, F32 only:
 *   laplace: out = mu + b (E1 - E2)    (two calls: E1 for every chain of a
 *                                       unit, then E2; b is the scale)
 *   weibull: out = lambda E^(1/k)      (scale lambda, shape k > 0)
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
brng_status brng_step_laplace(brng_ctx *ctx, const float *d_mu, const float *d_b, float *d_out);
brng_status brng_step_weibull(brng_ctx *ctx, const float *d_lambda, const float *d_k, float *d_out);

/* Poisson, a discrete getter (the expanded library of Sec. 3's future work):
 * one draw per chain from the uniform pool, computed in double precision;
 * d_lambda holds n_chains rates (float), d_out n_chains int32 counts.
 *   lambda < 10 : inversion, k = min{k : u <= F(k)}, one uniform;
 *   lambda >= 10: Hormann's transformed rejection with squeeze (PTRS), two
 *                 uniforms per attempt.
 * A unit's lanes take uniforms in rounds: one to every pending lane (lane
 * order), then one more to every pending lane with lambda >= 10.  lambda
 * outside [0, 2^30] (or NaN) gives -1 and takes nothing.  Layout CHAINS,
 * precision F32, U pool enabled.
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
brng_status brng_step_poisson(brng_ctx *ctx, const float *d_lambda, int32_t *d_out);

/* Binomial(n, p), the second discrete getter (the discrete library of Sec.
 * 3's future work): one draw per chain from the
 * uniform pool, computed in double precision; d_n holds n_chains trial
 * counts (int32), d_p n_chains probabilities (float), d_out n_chains int32
 * results.  With p' = min(p, 1 - p) the draw is made for p' and mirrored
 * (n - k) when p > 1/2:
 *   n p' < 10 : inversion, k = min{k : u <= F(k)}, one uniform;
 *   n p' >= 10: Hormann's transformed rejection with decomposition (BTRD):
 *               an attempt takes one uniform, or two when the first is
 *               above u_r v_r.
 * A unit's lanes take uniforms in rounds: one to every pending lane (lane
 * order), then one more to every pending lane that needs a second.  n < 0
 * or p outside [0, 1] (or NaN) gives -1 and takes nothing.  Layout CHAINS,
 * precision F32, U pool enabled.
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
brng_status brng_step_binomial(brng_ctx *ctx, const int32_t *d_n, const float *d_p, int32_t *d_out);

/* Multinomial(n, p) by conditional binomials (the discrete library of Sec.
 * 3's future work): one item per chain (n_chains items, layout CHAINS,
 * precision F32, U pool), item i with components [d_offsets[i],
 * d_offsets[i+1]) of d_w (float weights, need not add to 1) and d_out (int32
 * counts), d_n[i] trials.  x_k ~ Binomial(n - x_0 - ... - x_{k-1}, p_k / S_k)
 * for k < K - 1, x_{K-1} the rest; S_0 = p_0 + ... + p_{K-1} (index order,
 * double precision), S_{k+1} = S_k - p_k; S_k <= 0 gives probability 0, a
 * quotient above 1 is taken as 1.  Component k of every item that draws one
 * is one binomial call over the unit (as brng_step_binomial), k = 0, 1, ...
 * An item with n < 0, no components or a weight that is negative or not
 * finite gets -1 in every component and draws nothing.  d_offsets holds
 * n_chains + 1 nondecreasing entries from 0; d_w and d_out hold
 * d_offsets[n_chains] entries.
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
brng_status brng_step_multinomial(brng_ctx *ctx, const int32_t *d_offsets, const int32_t *d_n,
                                  const float *d_w, int32_t *d_out);

/* Dirichlet by normalised gammas (Sec. 1, footnote on Dirichlet): layout
 * ITEMS, item i has components [d_offsets[i], d_offsets[i+1]) of d_alpha and
 * d_out (F32).  Components are drawn in batches of 64, one gamma call per
 * batch.  n_items = n_chains of the context; d_offsets has n_items + 1
 * entries, starting at 0, each item 1..4096 components. */
brng_status brng_step_dirichlet(brng_ctx *ctx, const int32_t *d_offsets,
                                const float *d_alpha, float *d_out);

/* Full LDA on a corpus (the model whose Dirichlet redraws motivate the
 * method, Sec. 1 and its footnote), by the uncollapsed Gibbs sampler.  Per
 * sweep: phi_k ~ Dir(beta + n_k.) over the vocabulary for every topic,
 * theta_d ~ Dir(alpha + n_d.) for every document, then every token's topic
 * z ~ Cat(theta_d,k phi_k,w), one uniform per token in token order.  The
 * token draw quantises its fp32 weights p_k = theta_k phi_w,k against the
 * binade of their maximum, q_k = rint(p_k 2^(24 - e)) with max p = f 2^e,
 * f in [1/2, 1) (all 1 when max p = 0), and takes
 * the first k with t < q_0 + ... + q_k, t = (j Q) >> 23, Q the sum of the
 * q_k, j = (u 2^24 - 1) / 2.  Context: layout ITEMS, F32, kinds U, N, E
 * enabled, at least brng_lda_full_units(n_topics, n_vocab, n_docs) items.
 * A topic's vocabulary is cut into nb = ceil(n_vocab / BRNG_LDAF_VBLOCK)
 * blocks: the gammas of topic k's words [j BRNG_LDAF_VBLOCK,
 * (j + 1) BRNG_LDAF_VBLOCK) come from unit k nb + j, and phi_k divides them
 * by their sum over all blocks (the same Dirichlet: a gamma's law does not
 * depend on the stream that feeds it); document d is unit n_topics nb + d.
 * Every call continues those units' streams.
 * The state is the assignment d_z (int32 per token, in/out): a call first
 * recounts n_dk and n_kw from it (skipped with flags BRNG_LDAF_COUNTS_VALID,
 * when d_ndk and d_nkw already hold the counts of d_z, as a previous call
 * returned them), then runs `sweeps` sweeps; on return z,
 * n_dk ([n_docs][n_topics] int32) and n_kw ([n_topics][n_vocab] int32) are
 * consistent, and theta ([n_docs][n_topics]) and phi ([n_vocab][n_topics],
 * word-major: a token's topic weights are one row) hold the last sweep's
 * draws (float).  Tokens of document d are
 * [d_doc_offsets[d], d_doc_offsets[d+1]) clamped to [0, n_tokens); a word
 * id outside [0, n_vocab) gets z = -1, no count, and still takes its
 * uniform.  All arrays are caller-owned device memory.
 * Limits: 1 <= n_topics <= BRNG_LDAF_KMAX, 1 <= n_vocab <= BRNG_LDAF_VMAX,
 * alpha, beta > 0.  The token step takes one token per lane; up to 64
 * topics a lane keeps its weights in registers, above it forms them from
 * its phi row once for the largest, once for the total and once for the
 * count (the same topics either way).  Each topic block is
 * drawn by one wave (BRNG_LDAF_VBLOCK / 64 gamma rounds per sweep), beside
 * the documents' Dirichlets; with more than one block per topic a second
 * small kernel normalises phi.
 * Errors: BRNG_E_ARG (also for too few items), BRNG_E_KIND_DISABLED,
 * BRNG_E_UNSUPPORTED, BRNG_E_HIP. */
#define BRNG_LDAF_VMAX (1 << 20)
#define BRNG_LDAF_KMAX 1024
#define BRNG_LDAF_VBLOCK 1024
/* Items a full-LDA corpus uses: n_topics ceil(n_vocab / BRNG_LDAF_VBLOCK)
 * + n_docs (0 when n_vocab is 0). */
uint64_t brng_lda_full_units(uint32_t n_topics, uint32_t n_vocab, uint32_t n_docs);
typedef struct {
    uint32_t n_docs;
    uint32_t n_topics;
    uint32_t n_vocab;
    uint32_t sweeps;
    int32_t n_tokens;
    float alpha;               /* document-topic prior */
    float beta;                /* topic-word prior */
    uint32_t flags;            /* BRNG_LDAF_COUNTS_VALID or 0 */
    const int32_t *d_doc_offsets; /* n_docs + 1 token offsets */
    const int32_t *d_words;    /* word id per token */
    int32_t *d_z;              /* topic per token (in/out) */
    int32_t *d_ndk;            /* out: [n_docs][n_topics] */
    int32_t *d_nkw;            /* out: [n_topics][n_vocab] */
    float *d_theta;            /* out: [n_docs][n_topics] */
    float *d_phi;              /* out: [n_vocab][n_topics] */
} brng_lda_full_desc;
enum { BRNG_LDAF_COUNTS_VALID = 1u };
brng_status brng_run_lda_full(brng_ctx *ctx, const brng_lda_full_desc *h_desc);

/* ---------------------------------------------------------------------- */
/* Chain drivers (Fig. 1 generalised): many independent Gibbs chains, state */
/* in registers, one kernel for all steps.                                */
/* ---------------------------------------------------------------------- */
enum {
    BRNG_MODEL_TRIANGLE_F64 = 0, /* Eq. 1 / Fig. 1: x~U(0,1-y), y~U(0,1-x), fp64 */
    BRNG_MODEL_NORMEXP = 1,      /* s'~N(0.9 s, 0.5+|s|), e~Exp(1+s'^2), fp32 */
    BRNG_MODEL_GAMMA_CHAIN = 2,  /* g~Gamma(alpha,1), alpha' = 0.1 + g, fp32 */
    BRNG_MODEL_LDA = 3,          /* theta~Dir(0.1+counts), counts~Mult(n,theta) */
    BRNG_MODEL_EXP_CHAIN = 4,    /* e' ~ Exp(1 + e^2), fp32 */
    BRNG_NMODELS = 5
};
enum {
    BRNG_FLAG_RESUME = 1u /* continue from the units' cursors and d_state;
                             otherwise start fresh: cursors 0, windows
                             regenerated, model's initial state */
};

typedef struct {
    int32_t model;         /* BRNG_MODEL_* */
    uint32_t n_chains;     /* chains, or documents for LDA */
    uint32_t unit_base;    /* first context unit used; units are request-local
                              ids 0..n_units-1 for the Philox key */
    uint32_t flags;        /* BRNG_FLAG_* */
    uint64_t seed;         /* stream seed of this request */
    int32_t max_steps;     /* steps (sweeps for LDA) when d_steps is NULL */
    int32_t pad0;
    const int32_t *d_steps; /* per-chain steps (user order) or NULL */
    const int32_t *d_perm;  /* chains: slot -> chain, or NULL for identity
                               (see brng_sort_by_length); LDA: ignored (the
                               library schedules documents by their number
                               of components; results never depend on the
                               order) */
    void *d_state;          /* model state, user order, in/out:
                               TRIANGLE: double[2][n] (x then y)
                               NORMEXP : float[n] (s)
                               GAMMA   : float[n] (next shape alpha; alpha_0
                                         on a fresh start, must be > 0)
                               EXP     : float[n] (e; fresh: first E draw)
                               LDA     : int32 counts[total components] */
    void *d_trace;          /* [step][slot] first output, or NULL:
                               TRIANGLE x, NORMEXP s', GAMMA g, EXP e',
                               LDA theta ([sweep][component], float) */
    void *d_trace2;         /* second output, or NULL: TRIANGLE y, NORMEXP e,
                               LDA counts ([sweep][component], int32) */
    int64_t trace_stride;   /* elements between steps (>= n_chains; LDA: >=
                               total components) */
    const int32_t *d_offsets; /* LDA: n_docs + 1 component offsets */
    const int32_t *d_ntok;    /* LDA: tokens per document */
    double *d_sums;           /* per-chain summaries, or NULL: for each output
                                 its sum and its sum of squares over this
                                 call's steps, ADDED to what the array holds
                                 (zero it for a fresh total), user chain order:
                                 TRIANGLE double[4][n] (x, x^2, y, y^2),
                                 NORMEXP double[4][n] (s', s'^2, e, e^2),
                                 GAMMA and EXP double[2][n] (g or e', square),
                                 LDA double[2][total components] (theta,
                                 theta^2).  Each step adds (double)v and
                                 (double)v * (double)v in step order, so a run
                                 split over several calls (or served in
                                 slices) gives the same bits as one call */
} brng_gibbs_desc;

/* Requests one brng_run_gibbs call takes. */
#define BRNG_BATCH_MAX 4096

/* Run chains to completion on the context's stream: the one-at-a-time loop
 * of Sec. 1 (Eq. 1 / Fig. 1, the Dirichlet redraws of its footnote) for
 * many chains at once.  One request is one launch of its model's kernel (one
 * wave per unit, every step of every chain inside that launch).  Up to
 * BRNG_BATCH_MAX requests, of any models, run as one launch over all their
 * units (each wave runs its request's model), after small launches that copy
 * the requests' descriptors into the context's device table; the sequence
 * allocates nothing and can be captured in a graph.
 * Each request's units [unit_base, unit_base + n_units) must lie inside the
 * context and must not overlap another request's.  The needed kinds must be
 * enabled: TRIANGLE U64; NORMEXP N,E; GAMMA N,E; EXP E; LDA U,N,E.  LDA
 * documents need 1..256 components, a token count >= 0 and, with traces,
 * components inside trace_stride; a document that breaks this gets -1 in
 * every count of its state (when it has components) and nothing else.  A
 * single LDA request first runs a one-workgroup planning kernel that sorts
 * the documents by size (documents of up to 16 components share a wave,
 * each with its own streams), using the context's plan memory.  Traces
 * need max_steps rows of trace_stride elements.
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_HIP. */
brng_status brng_run_gibbs(brng_ctx *ctx, const brng_gibbs_desc *h_descs, uint32_t n_desc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * request run as brng_run_gibbs runs it on a context with these windows,
 * without a context.  Its unit records and pool windows live in a fixed
 * device array of BRNG_STATIC_SCRATCH_MB MiB that the library holds on each
 * GPU it runs on until the process ends; the call allocates nothing and
 * launches only the model's chain kernel on `hip_stream` (a hipStream_t, or
 * NULL for the default stream).  The request must start fresh (flags 0,
 * unit_base 0): every run draws from cursor 0 of its own streams, keyed by
 * (request-local unit, d->seed), so the results equal brng_run_gibbs on a
 * fresh context with window4.  window4[kind] as in brng_config (the model's
 * kinds must be enabled); wpb = waves per workgroup (1, 2, 4 or 8, halved
 * while a workgroup's LDS would exceed 64 KiB).  The footprint is, per kind
 * the model reads, n_units x window x entry size, plus 96 bytes per unit,
 * plus for LDA 4 x (8 + 6 n_docs) bytes of launch plan (each term rounded
 * up to 256 bytes); a request beyond the array returns
 * BRNG_E_TOO_LARGE.  Caller-owned device arrays as in brng_gibbs_desc.
 * Every call on one GPU uses the same array: calls that overlap on that GPU
 * (other streams, other threads) race and give undefined results; calls in
 * one stream's order are safe.  The array keeps the last call's contents,
 * which no later call reads.
 * Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_TOO_LARGE,
 * BRNG_E_UNSUPPORTED (device index above 63), BRNG_E_HIP. */
#define BRNG_STATIC_SCRATCH_MB 32
brng_status brng_run_gibbs_static(const brng_gibbs_desc *h_desc, const uint32_t *h_window4,
                                  int32_t wpb, void *hip_stream);

/* A scheduling aid with no counterpart in the paper.  Slot order for uneven
 * chain lengths: perm[p] = chain in slot p, chains
 * stably sorted by descending steps (so a unit's lanes finish together).
 * Host arrays of n entries.  Errors: BRNG_E_ARG. */
brng_status brng_sort_by_length(uint32_t n, const int32_t *h_steps, int32_t *h_perm);

/* The buffer counters of Sec. 2.2, one per unit and kind.  Copy the cursors
 * to the host as uint64[n_units][4] (waits for the
 * stream).  Errors: BRNG_E_ARG, BRNG_E_HIP. */
brng_status brng_get_cursors(brng_ctx *ctx, uint64_t *h_out);

/* Restore the buffer counters of Sec. 2.2 (checkpoint/resume, a library
 * addition): uint64[n_units][4]; invalidates the
 * windows, which the next call regenerates from the cursors.  Units keep
 * their stream keys.  Errors: BRNG_E_ARG, BRNG_E_HIP. */
brng_status brng_set_cursors(brng_ctx *ctx, const uint64_t *h_in);

/* The buffer contents of Sec. 2.2.  Copy unit `unit`'s current window of
 * `kind` to the host: *h_base gets the
 * pool index of its first entry, *h_len its valid length (0 if empty), and
 * h_out up to cap entries (float, or double for U64).  Waits for the
 * stream.  Errors: BRNG_E_ARG, BRNG_E_KIND_DISABLED, BRNG_E_HIP. */
brng_status brng_get_window(brng_ctx *ctx, int32_t kind, uint32_t unit, void *h_out,
                            uint32_t cap, uint64_t *h_base, uint32_t *h_len);

/* The conversion half of the core engine (the reducible base distributions
 * of Sec. 2.1) on caller-supplied words: n_words
 * 32-bit words (a multiple of 4, 16-byte aligned device arrays) become
 * n_words entries of kind U, N or E (floats; N pairs words 2i, 2i+1) or
 * n_words/2 entries of U64 (doubles), exactly as pool entries are made from
 * Philox words.  For validating the conversions and for callers with their
 * own word streams.  Asynchronous on `stream` (hipStream_t, NULL = default).
 * Errors: BRNG_E_ARG, BRNG_E_HIP. */
brng_status brng_convert(int32_t kind, const uint32_t *d_words, uint64_t n_words, void *d_out,
                         void *stream);

/* Context facts (a library aid, no passage of the paper): number of units
 * and the four window lengths (window4 holds 4 entries).  Host pointers;
 * either may be NULL.
 * Errors: BRNG_E_ARG. */
brng_status brng_get_info(const brng_ctx *ctx, uint32_t *n_units, uint32_t *window4);

/* Launch shape of the chain and step kernels (a tuning knob with no
 * counterpart in the paper; results do not
 * depend on it): waves per workgroup, 1, 2, 4 or 8; `reserved` must be 0.
 * Errors: BRNG_E_ARG. */
brng_status brng_set_launch(brng_ctx *ctx, int32_t waves_per_block, int32_t reserved);

/* Measurement support (no passage of the paper; for timing the chain
 * kernel alone, as the paper times its generators).  start_event and
 * stop_event are hipEvent_t handles the caller created with timing enabled
 * and owns.  The next brng_run_gibbs call in the plain form (one request)
 * launches its chain kernel, or the next brng_run_lda_full call with at
 * least one sweep its last sweep's document kernel, so that start_event is
 * recorded when the kernel starts and stop_event when it ends: their
 * elapsed time is the kernel's own
 * duration, without the dispatch gap that events recorded on the stream
 * around the call include.  The pair is used once and then forgotten; a
 * batched call leaves it pending.  Both NULL clears a pending pair.
 * Errors: BRNG_E_ARG (NULL ctx, or exactly one event NULL). */
brng_status brng_time_next_launch(brng_ctx *ctx, void *start_event, void *stop_event);

/* ---------------------------------------------------------------------- */
/* Served form: a request loop with continuous batching.  Requests (one    */
/* brng_gibbs_desc each) arrive at any time; the server admits them while  */
/* device memory within its budget and a slot are free, keeps their unit   */
/* tables and pools on the device, and advances every admitted request by  */
/* a time slice per tick, all admitted requests sharing one launch.  A     */
/* request's results do not depend on what else runs (its streams are its */
/* own: units keyed by (request-local unit id, request seed), Sec. 2.2's   */
/* buffers kept per request), so they equal a plain brng_run_gibbs of the  */
/* same request.  Suggested by the paper's asynchronous-service outlook    */
/* (Sec. 3).                                                               */
/* ---------------------------------------------------------------------- */
typedef struct brng_server brng_server;

typedef struct {
    uint64_t hbm_budget;  /* bytes of device memory for admitted requests'
                             unit tables and pools (counted per request:
                             its footprint), allocated once at open */
    uint32_t max_active;  /* requests admitted at once (slots), >= 1 */
    uint32_t tick_steps;  /* steps per tick for chain models, >= 1 */
    uint32_t tick_sweeps; /* sweeps per tick for LDA, >= 1 */
    uint32_t window[4];   /* pool window per unit per kind for every request
                             (as brng_config.window; kinds a model needs must
                             be non-zero) */
    uint32_t max_bypass_ms; /* while the oldest waiting request does not fit,
                               later ones that fit are admitted past it until
                               it has waited this long since its arrival
                               (0: strictly in submission order) */
    void *hip_stream;     /* hipStream_t for all server work, NULL = default */
} brng_serve_config;

typedef struct {
    uint64_t ticket;      /* from brng_serve_submit */
    uint64_t t_arrive_ns; /* arrival time given at submit (brng_serve_now) */
    uint64_t t_admit_ns;  /* when the server admitted it */
    uint64_t t_done_ns;   /* when the server saw its last tick complete */
    int32_t status;       /* BRNG_OK, or the error that ended it */
    int32_t pad;
} brng_serve_done;

typedef struct {
    uint32_t waiting;     /* submitted, not yet admitted */
    uint32_t active;      /* admitted, not finished */
    uint32_t ticks_in_flight;
    uint32_t pad;
    uint64_t bytes_in_use;   /* footprints of admitted requests */
    uint64_t bytes_peak;     /* largest bytes_in_use so far (<= hbm_budget) */
    uint64_t ticks;          /* ticks launched so far */
    uint64_t completed;      /* requests finished so far */
} brng_serve_stats;

/* Open a server: allocates the budget and creates its events.
 * Errors: BRNG_E_ARG, BRNG_E_NOMEM, BRNG_E_HIP; *out is NULL on error. */
brng_status brng_serve_open(const brng_serve_config *cfg, brng_server **out);

/* Steady-clock time in ns, the clock of the brng_serve_done stamps. */
uint64_t brng_serve_now(void);

/* Queue one request.  *h_desc is copied; unit_base must be 0 and flags 0
 * (a served request starts fresh: cursors 0, the model's initial state; for
 * GAMMA and LDA d_state holds alpha_0 / the initial counts).  Its device
 * arrays (state, steps, perm, traces, offsets, ntok) are the caller's and
 * must stay valid until the request is done; the state is updated in place.
 * t_arrive_ns is its arrival time (0: now).  Requests are admitted in
 * submission order, but a request that does not fit may be passed by later
 * ones for up to max_bypass_ms after its arrival (brng_serve_config).
 * Footprint = unit tables + pools of the kinds the model uses (plus one
 * int32 per chain slot for GAMMA).  Errors: BRNG_E_ARG (invalid request), BRNG_E_KIND_DISABLED (the
 * server's windows lack a kind the model needs), BRNG_E_NOMEM (footprint
 * above the whole budget: it could never be admitted). */
brng_status brng_serve_submit(brng_server *srv, const brng_gibbs_desc *h_desc,
                              uint64_t t_arrive_ns, uint64_t *ticket);

/* Do the server's work once: retire finished ticks (their finished requests
 * become done and free their memory), admit waiting requests that fit, and
 * launch the next tick when fewer than two are in flight.  wait = 1 blocks
 * until the oldest tick in flight has finished before retiring.
 * Errors: BRNG_E_ARG, BRNG_E_HIP. */
brng_status brng_serve_progress(brng_server *srv, int32_t wait);

/* Move up to `cap` finished requests, oldest first, to h_out; *n gets the
 * count.  Errors: BRNG_E_ARG. */
brng_status brng_serve_poll(brng_server *srv, brng_serve_done *h_out, uint32_t cap, uint32_t *n);

/* Copy the server's counters to *h_out (host).  Errors: BRNG_E_ARG. */
brng_status brng_serve_stats_get(const brng_server *srv, brng_serve_stats *h_out);

/* Finish every queued request, then free the server.  NULL is a no-op. */
brng_status brng_serve_close(brng_server *srv);

/* Integer status codes, in the style of the vector-library calls shown in
 * Sec. 1.  Human-readable status; never NULL. */
const char *brng_status_string(brng_status s);
/* hipError_t of the last BRNG_E_HIP in this thread (0 if none). */
int32_t brng_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BRNG_H */
