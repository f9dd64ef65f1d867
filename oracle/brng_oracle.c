/*
 * brng oracle: a plain, scalar, double-precision CPU reference for the
 * varying-parameter base-pool random number generator of Mahani & Sharabiani,
 * "Efficient SIMD RNG for Varying-Parameter Streams: C++ Class BatchRNG"
 * (arXiv 1412.4825).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product path never
 * does.  It shares no source, header, table or helper with the HIP library.
 *
 * Everything here is written for a reader holding the paper:
 *   - base pools of standard uniform, Gaussian and exponential deviates that
 *     are refilled in bulk and consumed one entry at a time, with a counter
 *     per pool (Sec. 2.1 "Key Concepts", Sec. 2.2 "Implementation");
 *   - reducible transforms a + (b - a) x (Sec. 2.1, second concept);
 *   - irreducible samplers built on the pools (Sec. 2.2, RNG functions);
 *   - the triangle Gibbs sampler (Eq. 1 and Fig. 1);
 *   - Dirichlet from normalised gammas (Sec. 1, footnote on Dirichlet).
 * The paper leaves the core generator, the Gaussian and exponential methods
 * and the gamma algorithm open; this file fixes them as follows:
 *   - core engine: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11);
 *   - Gaussian: Box-Muller (Box & Muller, 1958);
 *   - exponential: -ln u;
 *   - gamma: Marsaglia & Tsang (ACM TOMS 2000) with the u^(1/alpha) boost
 *     for alpha < 1, the uniform's logarithm taken from the exponential pool
 *     (ln u = -E, the paper's "logarithm of uniform deviates" buffer).
 *
 * Stream contract (what makes exact comparison possible):
 *   key     = (unit id, seed low 32 bits)
 *   counter = (block low 32, block high 32, kind, seed high 32)
 *   kinds   : 0 = U (fp32 uniform), 1 = N (Gaussian), 2 = E (exponential),
 *             3 = U64 (fp64 uniform)
 *   entry j of kind U/N/E lives in block j/4, word j%4; N pairs words
 *   (0,1) and (2,3) of a block with the cosine branch on the even entry;
 *   entry j of U64 uses words 2(j%2), 2(j%2)+1 of block j/2.
 *   A "call" gives one entry to every active slot of a unit, in ascending
 *   slot order; the pool counter (cursor) counts entries consumed.
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -o liboracle.so brng_oracle.c -lm
 * (-ffp-contract=off: every product and sum is rounded on its own, as
 * written, so the triangle trajectories are reproducible bit for bit).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_U = 0, OR_N = 1, OR_E = 2, OR_U64 = 3 };

/* ------------------------------------------------------------------------ */
/* Philox4x32 (Salmon et al. SC'11): round function and key schedule.       */
/* ------------------------------------------------------------------------ */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b; /* the full 64-bit product */
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* Apply `rounds` Philox4x32 rounds to ctr under key; rounds = 10 is the
 * generator.  The key is bumped by the Weyl constants between rounds, so the
 * first round uses the key as given. */
void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds,
                   uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < rounds; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The four words of pool block `block` for (seed, unit, kind). */
void or_block_words(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t block,
                    uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)block, (uint32_t)(block >> 32), kind,
                       (uint32_t)(seed >> 32)};
    uint32_t key[2] = {unit, (uint32_t)seed};
    or_philox4x32(ctr, key, 10, w);
}

/* ------------------------------------------------------------------------ */
/* Conversions to base deviates.                                            */
/* ------------------------------------------------------------------------ */

/* Uniform on the open midpoint grid (2k+1) 2^-24, k = the top 23 bits of w.
 * Every value is in (0,1), so the logarithm is finite and a + (b-a)u stays
 * strictly inside (a,b) (the paper writes U[0,1)). */
double or_u32(uint32_t w)
{
    uint64_t k = (uint64_t)(w >> 9);
    return (double)(2 * k + 1) * 0x1p-24;
}

/* Uniform on the grid (2k+1) 2^-53 with a 52-bit k built from two words. */
double or_u64(uint32_t wa, uint32_t wb)
{
    uint64_t k = ((uint64_t)wa << 20) | (uint64_t)(wb >> 12);
    return (double)(2 * k + 1) * 0x1p-53;
}

/* Entry j of the pool of `kind` for (seed, unit). */
double or_entry(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t j)
{
    uint32_t w[4];
    if (kind == OR_U64) {
        or_block_words(seed, unit, kind, j / 2, w);
        int p = (int)(j % 2);
        return or_u64(w[2 * p], w[2 * p + 1]);
    }
    or_block_words(seed, unit, kind, j / 4, w);
    int q = (int)(j % 4);
    if (kind == OR_U)
        return or_u32(w[q]);
    if (kind == OR_E)
        return -log(or_u32(w[q]));
    /* Box-Muller on the pair (w[2p], w[2p+1]). */
    int p = q / 2;
    double ua = or_u32(w[2 * p]);
    double ub = or_u32(w[2 * p + 1]);
    double r = sqrt(-2.0 * log(ua));
    double ang = 2.0 * M_PI * ub;
    return (q % 2 == 0) ? r * cos(ang) : r * sin(ang);
}

void or_entries(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t j0,
                uint64_t n, double *out)
{
    for (uint64_t i = 0; i < n; i++)
        out[i] = or_entry(seed, unit, kind, j0 + i);
}

/* Entries of `kind` made from caller-supplied words, as pool entries are made
 * from Philox words: U/E/N give one entry per word (N pairs words 2i, 2i+1),
 * U64 one entry per two words.  n_words is a multiple of 4. */
void or_convert(int kind, const uint32_t *w, uint64_t n_words, double *out)
{
    for (uint64_t i = 0; i < n_words; i += 2) {
        if (kind == OR_U64) {
            out[i / 2] = or_u64(w[i], w[i + 1]);
            continue;
        }
        for (int q = 0; q < 2; q++) {
            uint64_t j = i + (uint64_t)q;
            if (kind == OR_U)
                out[j] = or_u32(w[j]);
            else if (kind == OR_E)
                out[j] = -log(or_u32(w[j]));
            else {
                double r = sqrt(-2.0 * log(or_u32(w[i])));
                double ang = 2.0 * M_PI * or_u32(w[i + 1]);
                out[j] = q == 0 ? r * cos(ang) : r * sin(ang);
            }
        }
    }
}

/* Conversions of many words at once (for exhaustive checks). */
void or_u32_many(const uint32_t *w, uint64_t n, double *out)
{
    for (uint64_t i = 0; i < n; i++)
        out[i] = or_u32(w[i]);
}

void or_words(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t b0,
              uint64_t nb, uint32_t *out)
{
    for (uint64_t b = 0; b < nb; b++)
        or_block_words(seed, unit, kind, b0 + b, out + 4 * b);
}

/* ------------------------------------------------------------------------ */
/* Pool counters (Sec. 2.2: buffer_counter per reducible distribution).     */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t seed;
    uint32_t unit;
    uint64_t *cur; /* four counters, one per kind */
} stream_t;

static double take(stream_t *s, int kind)
{
    double v = or_entry(s->seed, s->unit, (uint32_t)kind, s->cur[kind]);
    s->cur[kind] += 1;
    return v;
}

/* ------------------------------------------------------------------------ */
/* Tolerances.  A single floating-point result r may differ from this       */
/* double-precision value by max(4 ulp32(M), 1e-6 M), where M is its        */
/* condition-aware magnitude.  For sums M is the largest of |r| and the     */
/* operands' magnitudes; for results that depend on a base deviate through  */
/* an amplifying map, M is |r| (1 + kappa) with kappa the relative          */
/* condition number with respect to that deviate.                           */
/* ------------------------------------------------------------------------ */

static double ulp32(double m)
{
    m = fabs(m);
    if (m < 0x1p-126)
        return 0x1p-149;
    int e;
    frexp(m, &e); /* m = f 2^e with f in [0.5,1) */
    return ldexp(1.0, e - 24);
}

double or_tol(double m)
{
    double a = 4.0 * ulp32(m), b = 1e-6 * fabs(m);
    return a > b ? a : b;
}

static double dmax(double a, double b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Reducible distributions (Sec. 2.1): one call over a set of chains.       */
/* Chains are grouped into units of `width` consecutive chains; cursors     */
/* holds four counters per unit.                                            */
/* ------------------------------------------------------------------------ */

static void unit_range(uint32_t n, uint32_t width, uint32_t u, uint32_t *lo,
                       uint32_t *hi)
{
    *lo = u * width;
    *hi = (*lo + width < n) ? *lo + width : n;
}

/* U(a,b) = a + (b - a) u */
void or_step_uniform(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, int kind,
                     uint64_t *cursors, const double *a, const double *b,
                     double *out, double *tol)
{
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            double x = take(&s, kind);
            double span = b[c] - a[c];
            out[c] = a[c] + span * x;
            if (tol)
                tol[c] = or_tol(dmax(fabs(out[c]), dmax(fabs(a[c]), fabs(span * x))));
        }
    }
}

/* N(mu, sigma) = mu + sigma z */
void or_step_normal(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                    const double *mu, const double *sigma, double *out,
                    double *tol)
{
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            double z = take(&s, OR_N);
            out[c] = mu[c] + sigma[c] * z;
            if (tol)
                tol[c] = or_tol(dmax(fabs(out[c]), dmax(fabs(mu[c]), fabs(sigma[c] * z))));
        }
    }
}

/* Exp(lambda) with rate lambda: E / lambda */
void or_step_exp(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                 const double *lambda, double *out, double *tol)
{
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            double e = take(&s, OR_E);
            out[c] = e / lambda[c];
            if (tol)
                tol[c] = or_tol(out[c]);
        }
    }
}

/* Laplace(mu, b) (GetLaplace, Sec. 2.2, built on the reducible functions):  */
/* mu + b (E1 - E2); the difference of two independent Exp(1) deviates is   */
/* standard Laplace.  Two calls on the exponential pool: E1 for every chain  */
/* of the unit, then E2 for every chain.                                    */
void or_step_laplace(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *mu, const double *b, double *out, double *tol)
{
    uint32_t nu = (n + width - 1) / width;
    if (width > 256) { /* units wider than the scratch row: not supported */
        for (uint32_t c = 0; c < n; c++) out[c] = NAN;
        return;
    }
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        double e1[256];
        for (uint32_t c = lo; c < hi; c++)
            e1[c - lo] = take(&s, OR_E);
        for (uint32_t c = lo; c < hi; c++) {
            double e2 = take(&s, OR_E);
            double p = b[c] * e1[c - lo], q = b[c] * e2;
            out[c] = mu[c] + (p - q);
            if (tol)
                tol[c] = or_tol(dmax(dmax(fabs(out[c]), fabs(mu[c])), dmax(fabs(p), fabs(q))));
        }
    }
}

/* Weibull(lambda, k) (GetWeibull, Sec. 2.2): lambda E^(1/k), one call on   */
/* the exponential pool.  The relative error of E and of the power grows    */
/* by (1 + |ln E|)/k, which the tolerance carries.                          */
void or_step_weibull(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *lambda, const double *k, double *out, double *tol)
{
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            double e = take(&s, OR_E);
            out[c] = lambda[c] * pow(e, 1.0 / k[c]);
            if (tol)
                tol[c] = or_tol(fabs(out[c]) * (1.0 + (1.0 + fabs(log(e))) / k[c]));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Gamma(alpha, 1): Marsaglia & Tsang (2000).                               */
/*                                                                          */
/* For a >= 1: d = a - 1/3, c = 1/sqrt(9d).  Draw x ~ N(0,1) and set        */
/* v = (1 + c x)^3; if 1 + c x <= 0 draw again.  Otherwise draw u and       */
/* accept d v when ln u < x^2/2 + d - d v + d ln v.  Here ln u = -E with E  */
/* from the exponential pool.  For alpha < 1 the draw is made with shape    */
/* alpha + 1 and multiplied by u'^(1/alpha) = exp(-E'/alpha).  A shape      */
/* outside (0, 2^64) has no draw: its value is NaN and it consumes nothing. */
/*                                                                          */
/* Consumption order: the slots of a unit share the pools and work in       */
/* rounds.  Each slot holds at most one draw.  In a round: a Gaussian for   */
/* every slot holding a draw with a valid shape (ascending slots); an       */
/* exponential for each of those whose 1 + c x > 0 (ascending); the accept  */
/* test; an exponential for every accepted draw with alpha < 1 (ascending); */
/* then, in ascending slot order, every slot whose draw is complete         */
/* (accepted, or with an invalid shape) hands its value on and takes its    */
/* next draw, if any.  So a slot whose draw is accepted starts its next     */
/* draw in the next round instead of waiting for the other slots.           */
/*                                                                          */
/* Besides the value the oracle reports, per draw:                          */
/*   tol    : bound on |gpu - oracle| (local rounding + the effect of an    */
/*            error bound `abound` carried by alpha itself),                */
/*   dg     : d g / d alpha (same base deviates),                           */
/*   margin : the smallest |decision value| / its tolerance over the        */
/*            draw's decisions (the sign of 1 + c x, the accept test and,  */
/*            for a shape with an error bound, alpha < 1); a value <= 1    */
/*            means an fp32 implementation may decide the other way,       */
/*   nN, nE : entries consumed,                                             */
/*   r0, r1 : the rounds (counted from 0 in this call) in which the draw    */
/*            started and completed; a flip changes consumption from the  */
/*            round it is made in, anywhere in [r0, r1].                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double g, tol, dg, margin;
    int nN, nE;
    int r0, r1; /* rounds of the draw's first Gaussian and of its completion */
} gdraw_t;

/* q(y) = 3 ln(1+y) - 3y + 3y^2/2 - y^3; d q(y) is the accept statistic
 * x^2/2 + d(1 - v + ln v) rewritten with y = c x (used here only for the
 * tolerance scales, never for a decision). */
static double qfun(double y) { return 3.0 * log1p(y) - 3.0 * y + 1.5 * y * y - y * y * y; }

#define OR_MAXSLOT 256

/* Where the draws of a unit come from and where they go. */
typedef struct gsrc gsrc_t;
struct gsrc {
    /* give slot k its next draw: 1 and the shape (and its error bound), or 0 */
    int (*next)(gsrc_t *g, int k, double *alpha, double *abound);
    /* slot k's draw is complete */
    void (*done)(gsrc_t *g, int k, const gdraw_t *r);
    void *ctx;
};

static int shape_ok(double a) { return a > 0.0 && a < 0x1p64; }

static void or_gamma_rounds(stream_t *s, int nslots, gsrc_t *src)
{
    double alpha[OR_MAXSLOT], ab[OR_MAXSLOT], d[OR_MAXSLOT], c[OR_MAXSLOT];
    double x[OR_MAXSLOT], v0[OR_MAXSLOT];
    double kx[OR_MAXSLOT]; /* |d ln(g)/d ln(x)| of the accepted draw */
    uint8_t hold[OR_MAXSLOT], acc[OR_MAXSLOT];
    gdraw_t res[OR_MAXSLOT];
    int any = 0, rnd = 0;
    for (int k = 0; k < nslots; k++) {
        hold[k] = (uint8_t)src->next(src, k, &alpha[k], &ab[k]);
        any |= hold[k];
    }
    /* per-draw setup */
#define SETUP(k, r)                                                              \
    do {                                                                         \
        res[k].g = 0.0; res[k].tol = 0.0; res[k].dg = 0.0;                      \
        res[k].margin = INFINITY; res[k].nN = 0; res[k].nE = 0;                  \
        res[k].r0 = (r); res[k].r1 = -1;                                         \
        kx[k] = 0.0;                                                             \
        if (shape_ok(alpha[k])) {                                                \
            double a_ = alpha[k] < 1.0 ? alpha[k] + 1.0 : alpha[k];              \
            d[k] = a_ - 1.0 / 3.0;                                               \
            c[k] = 1.0 / sqrt(9.0 * d[k]);                                       \
            /* alpha < 1 (the boost) is a decision too when alpha carries   */  \
            /* an error bound */                                                \
            if (ab[k] > 0.0)                                                     \
                res[k].margin = fabs(alpha[k] - 1.0) / ab[k];                    \
        }                                                                        \
    } while (0)
    for (int k = 0; k < nslots; k++)
        if (hold[k])
            SETUP(k, 0);
    while (any) {
        /* a Gaussian for every slot holding a valid draw, ascending */
        for (int k = 0; k < nslots; k++) {
            acc[k] = 0;
            if (!hold[k] || !shape_ok(alpha[k]))
                continue;
            x[k] = take(s, OR_N);
            res[k].nN++;
            v0[k] = 1.0 + c[k] * x[k];
            /* sign decision on 1 + c x */
            double y = c[k] * x[k];
            double t = or_tol(dmax(1.0, fabs(y))) + fabs(y / (2.0 * d[k])) * ab[k];
            double m = fabs(v0[k]) / t;
            if (m < res[k].margin)
                res[k].margin = m;
        }
        /* an exponential for each of those with 1 + c x > 0, ascending */
        for (int k = 0; k < nslots; k++) {
            if (!hold[k] || !shape_ok(alpha[k]) || !(v0[k] > 0.0))
                continue;
            double e = take(s, OR_E);
            res[k].nE++;
            double v = v0[k] * v0[k] * v0[k];
            double stat = e + (0.5 * x[k] * x[k] + d[k] - d[k] * v + d[k] * log(v));
            /* decision tolerance: representation of the base deviates
             * (E, and x through y), plus alpha's own error bound */
            double y = c[k] * x[k];
            double dq = d[k] * qfun(y);
            double cond = d[k] * 3.0 * pow(y, 4) / (1.0 + y);
            double dstat = qfun(y) + 1.5 * pow(y, 4) / (1.0 + y);
            double t = or_tol(e + fabs(dq) + fabs(cond)) + fabs(dstat) * ab[k];
            double m = fabs(stat) / t;
            if (m < res[k].margin)
                res[k].margin = m;
            if (stat > 0.0) { /* ln u = -E < x^2/2 + d(1 - v + ln v) */
                acc[k] = 1;
                res[k].g = d[k] * v;
                kx[k] = fabs(3.0 * y / (1.0 + y));
                res[k].dg = (1.0 + y) * (1.0 + y) * (1.0 - 0.5 * y);
                res[k].tol = or_tol(res[k].g * (1.0 + kx[k])) + fabs(res[k].dg) * ab[k];
            }
        }
        /* the boost for accepted draws with alpha < 1, ascending */
        for (int k = 0; k < nslots; k++) {
            if (!acc[k] || !(alpha[k] < 1.0))
                continue;
            double e = take(s, OR_E);
            res[k].nE++;
            double f = exp(-e / alpha[k]);
            double g1 = res[k].g;
            double dg1 = res[k].dg;
            res[k].g = g1 * f;
            res[k].dg = f * dg1 + res[k].g * e / (alpha[k] * alpha[k]);
            double kappa = kx[k] + e / alpha[k];
            res[k].tol = or_tol(res[k].g * (1.0 + kappa)) + fabs(res[k].dg) * ab[k];
        }
        /* complete draws hand on their value and take the next, ascending */
        any = 0;
        for (int k = 0; k < nslots; k++) {
            if (hold[k] && (acc[k] || !shape_ok(alpha[k]))) {
                if (!shape_ok(alpha[k]))
                    res[k].g = NAN;
                res[k].r1 = rnd;
                src->done(src, k, &res[k]);
                hold[k] = (uint8_t)src->next(src, k, &alpha[k], &ab[k]);
                if (hold[k])
                    SETUP(k, rnd + 1);
            }
            any |= hold[k];
        }
        rnd++;
    }
#undef SETUP
}

/* One draw per slot (the one-at-a-time call). */
typedef struct {
    const double *alpha;
    uint8_t *given;
    gdraw_t *out;
} one_each_t;

static int one_each_next(gsrc_t *g, int k, double *alpha, double *abound)
{
    one_each_t *o = (one_each_t *)g->ctx;
    if (o->given[k])
        return 0;
    o->given[k] = 1;
    *alpha = o->alpha[k];
    *abound = 0.0;
    return 1;
}

static void one_each_done(gsrc_t *g, int k, const gdraw_t *r)
{
    ((one_each_t *)g->ctx)->out[k] = *r;
}

/* One gamma draw per chain, chains grouped into units of `width`. */
void or_step_gamma(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                   const double *alpha, double *out, double *tol, double *margin,
                   int32_t *nN, int32_t *nE)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    uint8_t given[OR_MAXSLOT];
    gdraw_t res[OR_MAXSLOT];
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        int ns = (int)(hi - lo);
        memset(given, 0, sizeof(given));
        one_each_t o = {alpha + lo, given, res};
        gsrc_t src = {one_each_next, one_each_done, &o};
        or_gamma_rounds(&s, ns, &src);
        for (int k = 0; k < ns; k++) {
            out[lo + k] = res[k].g;
            if (tol) tol[lo + k] = res[k].tol;
            if (margin) margin[lo + k] = res[k].margin;
            if (nN) nN[lo + k] = res[k].nN;
            if (nE) nE[lo + k] = res[k].nE;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Dirichlet (Sec. 1, footnote): y_k ~ Gamma(alpha_k, 1), x_k = y_k / sum.  */
/* One item (a unit) holds K components, drawn by 64 slots in gamma rounds: */
/* the slots start with components 0..63, and a slot whose draw completes   */
/* takes the lowest component not yet started.                             */
/* ------------------------------------------------------------------------ */

#define OR_BATCH 64

typedef struct {
    int K, next;
    const double *alpha;
    int comp[OR_BATCH];
    double *y, *ytol, mmin;
} comps_t;

static int comps_next(gsrc_t *g, int k, double *alpha, double *abound)
{
    comps_t *c = (comps_t *)g->ctx;
    if (c->next >= c->K)
        return 0;
    c->comp[k] = c->next++;
    *alpha = c->alpha[c->comp[k]];
    *abound = 0.0;
    return 1;
}

static void comps_done(gsrc_t *g, int k, const gdraw_t *r)
{
    comps_t *c = (comps_t *)g->ctx;
    c->y[c->comp[k]] = r->g;
    c->ytol[c->comp[k]] = r->tol;
    if (r->margin < c->mmin)
        c->mmin = r->margin;
}

/* The K gammas y_k ~ Gamma(alpha_k, 1) of one unit, with their tolerances;
 * returns the smallest decision margin. */
static double gamma_comps(stream_t *s, int K, const double *alpha, double *y, double *ytol)
{
    comps_t cs;
    cs.K = K;
    cs.next = 0;
    cs.alpha = alpha;
    cs.y = y;
    cs.ytol = ytol;
    cs.mmin = INFINITY;
    gsrc_t src = {comps_next, comps_done, &cs};
    or_gamma_rounds(s, OR_BATCH, &src);
    return cs.mmin;
}

/* theta_k = y_k / sum y, with tol (when non-NULL) a bound on |gpu theta -
 * oracle theta| for fp32 gammas summed in fp32. */
static void dirichlet_normalize(int K, const double *y, const double *ytol, double *theta,
                                double *tol)
{
    double S = 0.0, St = 0.0;
    for (int k = 0; k < K; k++) {
        S += y[k];
        St += ytol[k];
    }
    for (int k = 0; k < K; k++) {
        theta[k] = (S > 0.0) ? y[k] / S : 0.0;
        if (tol) {
            /* relative error of y_k plus that of the sum (including an fp32
             * summation of K terms) */
            double rel = (y[k] > 0.0 ? ytol[k] / y[k] : 0.0) +
                         (S > 0.0 ? St / S : 0.0) + (double)K * 0x1p-24;
            tol[k] = or_tol(theta[k]) + theta[k] * rel;
            if (y[k] < 0x1p-126) /* an underflowed gamma gives theta ~ 0 */
                tol[k] = dmax(tol[k], 0x1p-126 / (S > 0.0 ? S : 1.0));
        }
    }
}

/* Draw theta for one item; y/ytol are scratch of length K. Returns the
 * smallest decision margin. tol: bound on |gpu theta - oracle theta|. */
static double dirichlet_item(stream_t *s, int K, const double *alpha,
                             double *theta, double *tol, double *y, double *ytol)
{
    const double mmin = gamma_comps(s, K, alpha, y, ytol);
    dirichlet_normalize(K, y, ytol, theta, tol);
    return mmin;
}

/* ------------------------------------------------------------------------ */
/* Poisson(lambda): a discrete getter (the expanded library of Sec. 3's     */
/* future work).  Double precision on both sides; the U pool only.          */
/*                                                                          */
/*   lambda < 10: inversion with one uniform, k = min{k : u <= F(k)}, where */
/*     F is accumulated from p_0 = exp(-lambda), p_k = p_{k-1} lambda / k.  */
/*   lambda >= 10: transformed rejection with squeeze (Hormann 1993,        */
/*     "PTRS"): an attempt takes two uniforms u, v; with U = u - 1/2,       */
/*     us = 1/2 - |U|, k = floor((2a/us + b) U + lambda + 0.43); accept at  */
/*     once if us >= 0.07 and v <= v_r; reject if k < 0 or (us < 0.013 and */
/*     v > us); otherwise accept iff                                       */
/*       ln v + ln(inv_alpha) - ln(a/us^2 + b)                               */
/*         <= -lambda + k ln(lambda) - ln Gamma(k + 1),                      */
/*     with b = 0.931 + 2.53 sqrt(lambda), a = -0.059 + 0.02483 b,           */
/*     inv_alpha = 1.1239 + 1.1328/(b - 3.4), v_r = 0.9277 - 3.6224/(b - 2). */
/*   lambda outside [0, 2^30] (or NaN): result -1, nothing consumed.        */
/*                                                                          */
/* Consumption order (the slots of a unit share the U pool, in rounds):     */
/* in each round one uniform to every slot still pending (ascending), then  */
/* one more to every pending slot with lambda >= 10 (ascending); a slot     */
/* with lambda < 10 is pending only in round 0.                             */
/*                                                                          */
/* margin: the smallest |decision value| / its tolerance over the draw's    */
/* decisions whose operands are not exact (u against F(k); the floor; v     */
/* against v_r; the final test); <= 1 means a double-precision              */
/* implementation with other elementary functions may decide otherwise.    */
/* ------------------------------------------------------------------------ */

#define OR_POIS_SMALL 10.0
#define OR_POIS_MAX 0x1p30

static int pois_valid(double lam) { return lam >= 0.0 && lam <= OR_POIS_MAX; }

/* inversion with the uniform u; *margin receives the decisions' margin */
static int32_t pois_invert(double lam, double u, double *margin)
{
    double p = exp(-lam), F = p, m = INFINITY;
    int32_t k = 0;
    for (;;) {
        double t = 0x1p-46 * (double)(k + 1);
        double mk = fabs(u - F) / t;
        if (mk < m) m = mk;
        if (u <= F || k >= 1000)
            break;
        k += 1;
        p = p * lam / (double)k;
        F = F + p;
    }
    *margin = m;
    return k;
}

typedef struct {
    double lam, slam, loglam, a, b, invalpha, vr;
} ptrs_t;

static void ptrs_setup(ptrs_t *P, double lam)
{
    P->lam = lam;
    P->slam = sqrt(lam);
    P->loglam = log(lam);
    P->b = 0.931 + 2.53 * P->slam;
    P->a = -0.059 + 0.02483 * P->b;
    P->invalpha = 1.1239 + 1.1328 / (P->b - 3.4);
    P->vr = 0.9277 - 3.6224 / (P->b - 2.0);
}

/* one attempt: 1 = accept with *k, 0 = reject; *margin is lowered */
static int ptrs_attempt(const ptrs_t *P, double u, double v, int32_t *k, double *margin)
{
    double U = u - 0.5;
    double us = 0.5 - fabs(U);
    double slope = 2.0 * P->a / us + P->b;
    double x = slope * U + P->lam + 0.43;
    double fl = floor(x);
    double d = fmin(x - fl, fl + 1.0 - x);
    double tx = 0x1p-46 * (fabs(slope * U) + P->lam + 1.0);
    if (d / tx < *margin) *margin = d / tx;
    double kk = fl;
    if (us >= 0.07) {
        double mv = fabs(v - P->vr) / 0x1p-48;
        if (mv < *margin) *margin = mv;
        if (v <= P->vr) {
            *k = (int32_t)kk;
            return 1;
        }
    }
    if (kk < 0.0 || (us < 0.013 && v > us))
        return 0;
    double q = P->a / (us * us) + P->b;
    double lhs = log(v) + log(P->invalpha) - log(q);
    double lg = lgamma(kk + 1.0);
    double rhs = -P->lam + kk * P->loglam - lg;
    double t = 0x1p-44 * (fabs(log(v)) + fabs(log(P->invalpha)) + fabs(log(q)) + P->lam +
                          fabs(kk * P->loglam) + fabs(lg) + 1.0);
    double mt = fabs(lhs - rhs) / t;
    if (mt < *margin) *margin = mt;
    if (lhs <= rhs) {
        *k = (int32_t)kk;
        return 1;
    }
    return 0;
}

void or_step_poisson(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *lambda, int32_t *out, double *margin)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    uint8_t pend[OR_MAXSLOT];
    double u1[OR_MAXSLOT];
    ptrs_t P[OR_MAXSLOT];
    for (uint32_t un = 0; un < nu; un++) {
        stream_t s = {seed, unit0 + un, cursors + 4 * (size_t)un};
        uint32_t lo, hi;
        unit_range(n, width, un, &lo, &hi);
        int ns = (int)(hi - lo), any = 0;
        for (int k = 0; k < ns; k++) {
            double lam = lambda[lo + k];
            pend[k] = (uint8_t)pois_valid(lam);
            out[lo + k] = -1;
            if (margin) margin[lo + k] = INFINITY;
            if (pend[k] && lam >= OR_POIS_SMALL)
                ptrs_setup(&P[k], lam);
            any |= pend[k];
        }
        for (int round = 0; any && round < 1 << 20; round++) {
            for (int k = 0; k < ns; k++)
                if (pend[k])
                    u1[k] = take(&s, OR_U);
            for (int k = 0; k < ns; k++) {
                if (!pend[k])
                    continue;
                double lam = lambda[lo + k];
                double m = margin ? margin[lo + k] : INFINITY;
                if (lam < OR_POIS_SMALL) {
                    double mi;
                    out[lo + k] = pois_invert(lam, u1[k], &mi);
                    if (mi < m) m = mi;
                    pend[k] = 0;
                } else {
                    double v = take(&s, OR_U);
                    int32_t kk;
                    if (ptrs_attempt(&P[k], u1[k], v, &kk, &m)) {
                        out[lo + k] = kk;
                        pend[k] = 0;
                    }
                }
                if (margin) margin[lo + k] = m;
            }
            any = 0;
            for (int k = 0; k < ns; k++)
                any |= pend[k];
        }
    }
}


/* ------------------------------------------------------------------------ */
/* Binomial(n, p): the second discrete getter (Sec. 3's future work).       */
/* Double precision; the U pool only.  With p' = min(p, 1 - p) the draw is  */
/* made for p' and mirrored (n - k) when p > 1/2.                           */
/*                                                                          */
/*   n p' < 10: inversion with one uniform, k = min{k : u <= F(k)}, F       */
/*     accumulated from P_0 = exp(n ln(1 - p')),                            */
/*     P_k = P_{k-1} (n - k + 1) / k * (p'/(1 - p')), k <= n.               */
/*   n p' >= 10: transformed rejection with decomposition (Hormann 1993,    */
/*     "BTRD").  Setup: m = floor((n + 1) p'), spq = sqrt(n p' q'),         */
/*     b = 1.15 + 2.53 spq, a = -0.0873 + 0.0248 b + 0.01 p',               */
/*     c = n p' + 0.5, alpha = (2.83 + 5.1/b) spq, v_r = 0.92 - 4.2/b,      */
/*     u_r v_r = 0.86 v_r.  An attempt takes a first uniform v:             */
/*       v <= u_r v_r: U = v/v_r - 0.43, k = floor((2a/(1/2 - |U|) + b) U   */
/*         + c), accepted at once (if 0 <= k <= n);                         */
/*       otherwise a second uniform w: if v >= v_r, U = w - 1/2 and V = v;  */
/*         else U = v/v_r - 0.93, U = sign(U)/2 - U, V = w v_r;             */
/*         us = 1/2 - |U|, k = floor((2a/us + b) U + c), rejected unless    */
/*         0 <= k <= n, and accepted iff                                    */
/*           ln(V alpha / (a/us^2 + b)) <= ln P(k) - ln P(m)                */
/*         (the method's exact test, evaluated with ln Gamma).              */
/*   n < 0, p outside [0, 1] or NaN: result -1, nothing consumed.           */
/*                                                                          */
/* Consumption order, in rounds over a unit's slots: one uniform to every   */
/* pending slot (ascending), then one more to every pending slot on the     */
/* rejection path whose first uniform was above u_r v_r (ascending); an     */
/* inversion slot is pending only in round 0.                               */
/* margin: as for Poisson, over the decisions with inexact operands.        */
/* ------------------------------------------------------------------------ */

static int32_t binom_invert(int32_t n, double pp, double u, double *margin)
{
    double q = 1.0 - pp, s = pp / q;
    double P = exp((double)n * log1p(-pp)), F = P, mm = INFINITY;
    int32_t k = 0;
    for (;;) {
        double mk = fabs(u - F) / (0x1p-46 * (double)(k + 1));
        if (mk < mm) mm = mk;
        if (u <= F || k >= n)
            break;
        k += 1;
        P = P * (double)(n - k + 1) / (double)k * s;
        F = F + P;
    }
    *margin = mm;
    return k;
}

typedef struct {
    double n, p, lp_m, logp, logq, lgn1, a, b, c, alpha, vr, urvr;
    int32_t ni, m;
} btrd_t;

static double binom_lp(const btrd_t *B, double k)
{
    return B->lgn1 - lgamma(k + 1.0) - lgamma(B->n - k + 1.0) + k * B->logp + (B->n - k) * B->logq;
}

static void btrd_setup(btrd_t *B, int32_t n, double pp)
{
    B->ni = n;
    B->n = (double)n;
    B->p = pp;
    double q = 1.0 - pp;
    B->m = (int32_t)floor((B->n + 1.0) * pp);
    double spq = sqrt(B->n * pp * q);
    B->b = 1.15 + 2.53 * spq;
    B->a = -0.0873 + 0.0248 * B->b + 0.01 * pp;
    B->c = B->n * pp + 0.5;
    B->alpha = (2.83 + 5.1 / B->b) * spq;
    B->vr = 0.92 - 4.2 / B->b;
    B->urvr = 0.86 * B->vr;
    B->logp = log(pp);
    B->logq = log1p(-pp);
    B->lgn1 = lgamma(B->n + 1.0);
    B->lp_m = binom_lp(B, (double)B->m);
}

static void lower(double *m, double v) { if (v < *m) *m = v; }

/* distance of x to the nearest integer, over its rounding scale */
static double floor_margin(double x, double scale)
{
    double fl = floor(x);
    return fmin(x - fl, fl + 1.0 - x) / (0x1p-46 * (scale + 1.0));
}

/* first part of an attempt: 1 = accepted at once with *k, 0 = needs w */
static int btrd_first(const btrd_t *B, double v, int32_t *k, double *margin)
{
    lower(margin, fabs(v - B->urvr) / 0x1p-48);
    if (v <= B->urvr) {
        double U = v / B->vr - 0.43;
        double t = (2.0 * B->a / (0.5 - fabs(U)) + B->b) * U;
        double x = t + B->c;
        lower(margin, floor_margin(x, fabs(t) + B->c));
        double kk = floor(x);
        if (kk >= 0.0 && kk <= B->n) {
            *k = (int32_t)kk;
            return 1;
        }
        return -1; /* outside [0, n]: the attempt is rejected */
    }
    return 0;
}

/* second part: 1 = accept with *k, 0 = reject */
static int btrd_second(const btrd_t *B, double v, double w, int32_t *k, double *margin)
{
    double U, V;
    lower(margin, fabs(v - B->vr) / 0x1p-48);
    if (v >= B->vr) {
        U = w - 0.5;
        V = v;
    } else {
        U = v / B->vr - 0.93;
        U = (U >= 0.0 ? 0.5 : -0.5) - U;
        V = w * B->vr;
    }
    double us = 0.5 - fabs(U);
    double t = (2.0 * B->a / us + B->b) * U;
    double x = t + B->c;
    if (!(x >= 0.0 && x < B->n + 1.0)) /* k < 0 or k > n (also x NaN/inf) */
        return 0;
    lower(margin, floor_margin(x, fabs(t) + B->c));
    double kk = floor(x);
    double lhs = log(V * B->alpha / (B->a / (us * us) + B->b));
    double lpk = binom_lp(B, kk);
    double rhs = lpk - B->lp_m;
    double tol = 0x1p-44 * (fabs(lhs) + fabs(lpk) + fabs(B->lp_m) + B->lgn1 + 1.0);
    lower(margin, fabs(lhs - rhs) / tol);
    if (lhs <= rhs) {
        *k = (int32_t)kk;
        return 1;
    }
    return 0;
}

/* One binomial call over a unit's slots: every slot k with act[k] draws
 * Binomial(n[k], p[k]) (as above; -1 for invalid parameters); other slots
 * are left alone.  margin[k] is lowered by the draw's decisions. */
static void binom_call(stream_t *s, int ns, const int32_t *nn, const double *pr,
                       const uint8_t *act, int32_t *out, double *margin)
{
    uint8_t pend[OR_MAXSLOT], flip[OR_MAXSLOT], inv[OR_MAXSLOT];
    double v1[OR_MAXSLOT], pp[OR_MAXSLOT];
    btrd_t B[OR_MAXSLOT];
    int any = 0;
    for (int k = 0; k < ns; k++) {
        pend[k] = 0;
        if (!act[k])
            continue;
        int32_t n = nn[k];
        double p = pr[k];
        out[k] = -1;
        pend[k] = (uint8_t)(n >= 0 && p >= 0.0 && p <= 1.0);
        if (!pend[k])
            continue;
        flip[k] = (uint8_t)(p > 0.5);
        pp[k] = flip[k] ? 1.0 - p : p;
        inv[k] = (uint8_t)((double)n * pp[k] < 10.0);
        if (!inv[k])
            btrd_setup(&B[k], n, pp[k]);
        any = 1;
    }
    for (int round = 0; any && round < 1 << 20; round++) {
        for (int k = 0; k < ns; k++)
            if (pend[k])
                v1[k] = take(s, OR_U);
        for (int k = 0; k < ns; k++) {
            if (!pend[k])
                continue;
            double mg = margin ? margin[k] : INFINITY;
            int32_t kk = 0, done = 0;
            if (inv[k]) {
                double mi;
                kk = binom_invert(nn[k], pp[k], v1[k], &mi);
                lower(&mg, mi);
                done = 1;
            } else {
                int r = btrd_first(&B[k], v1[k], &kk, &mg);
                if (r == 1) {
                    done = 1;
                } else if (r == 0) {
                    double w = take(s, OR_U);
                    done = btrd_second(&B[k], v1[k], w, &kk, &mg);
                }
            }
            if (done) {
                out[k] = flip[k] ? nn[k] - kk : kk;
                pend[k] = 0;
            }
            if (margin) margin[k] = mg;
        }
        any = 0;
        for (int k = 0; k < ns; k++)
            any |= pend[k];
    }
}

void or_step_binomial(uint64_t seed, uint32_t unit0, uint32_t n_ch, uint32_t width,
                      uint64_t *cursors, const int32_t *nn, const double *pr, int32_t *out,
                      double *margin)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n_ch + width - 1) / width;
    uint8_t act[OR_MAXSLOT];
    memset(act, 1, sizeof(act));
    for (uint32_t un = 0; un < nu; un++) {
        stream_t s = {seed, unit0 + un, cursors + 4 * (size_t)un};
        uint32_t lo, hi;
        unit_range(n_ch, width, un, &lo, &hi);
        if (margin)
            for (uint32_t c = lo; c < hi; c++) margin[c] = INFINITY;
        binom_call(&s, (int)(hi - lo), nn + lo, pr + lo, act, out + lo, margin ? margin + lo : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Multinomial(n, p_0..p_{K-1}) by conditional binomials (the discrete       */
/* library of Sec. 3's future work): x_k ~ Binomial(n - x_0 - ... - x_{k-1},  */
/* p_k / S_k) for k < K - 1, x_{K-1} the rest, where S_k is the weight left:  */
/* S_0 = p_0 + ... + p_{K-1} summed in index order and S_{k+1} = S_k - p_k, */
/* in double precision; S_k <= 0 gives probability 0, a quotient above 1 is */
/* taken as 1.  Items are the */
/* chains of a unit (one item per slot, components by offsets).  Component  */
/* k of every item that draws one (k < K_i - 1) is one binomial call over    */
/* the unit, k = 0, 1, ...  An item with n < 0, K < 1 or a weight that is   */
/* negative or not finite gives -1 in all its components and draws nothing. */
/* ------------------------------------------------------------------------ */
void or_step_multinomial(uint64_t seed, uint32_t unit0, uint32_t n_items, uint32_t width,
                         uint64_t *cursors, const int32_t *offsets, const int32_t *nn,
                         const double *pw, int32_t *out, double *margin)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n_items + width - 1) / width;
    for (uint32_t un = 0; un < nu; un++) {
        stream_t s = {seed, unit0 + un, cursors + 4 * (size_t)un};
        uint32_t lo, hi;
        unit_range(n_items, width, un, &lo, &hi);
        int ns = (int)(hi - lo), kmax = 0;
        uint8_t ok[OR_MAXSLOT], act[OR_MAXSLOT];
        int32_t rem[OR_MAXSLOT], x[OR_MAXSLOT];
        double pk[OR_MAXSLOT], mg[OR_MAXSLOT];
        for (int j = 0; j < ns; j++) {
            uint32_t i = lo + (uint32_t)j;
            int32_t K = offsets[i + 1] - offsets[i];
            int good = nn[i] >= 0 && K >= 1;
            for (int32_t c = 0; good && c < K; c++) {
                double w = pw[offsets[i] + c];
                good = w >= 0.0 && w < INFINITY;
            }
            ok[j] = (uint8_t)good;
            rem[j] = nn[i];
            mg[j] = INFINITY;
            for (int32_t c = 0; c < K; c++)
                out[offsets[i] + c] = -1;
            if (good && K > kmax)
                kmax = K;
        }
        double S[OR_MAXSLOT];
        for (int j = 0; j < ns; j++) {
            uint32_t i = lo + (uint32_t)j;
            int32_t K = offsets[i + 1] - offsets[i];
            S[j] = 0.0;
            for (int32_t c = 0; ok[j] && c < K; c++)
                S[j] += pw[offsets[i] + c];
        }
        for (int32_t k = 0; k + 1 < kmax; k++) {
            for (int j = 0; j < ns; j++) {
                uint32_t i = lo + (uint32_t)j;
                int32_t K = offsets[i + 1] - offsets[i];
                act[j] = (uint8_t)(ok[j] && k + 1 < K);
                if (!act[j])
                    continue;
                double w = pw[offsets[i] + k];
                double q = S[j] > 0.0 ? w / S[j] : 0.0;
                pk[j] = q > 1.0 ? 1.0 : q;
                S[j] -= w;
            }
            binom_call(&s, ns, rem, pk, act, x, mg);
            for (int j = 0; j < ns; j++) {
                if (!act[j])
                    continue;
                uint32_t i = lo + (uint32_t)j;
                out[offsets[i] + k] = x[j];
                rem[j] -= x[j];
            }
        }
        for (int j = 0; j < ns; j++) {
            uint32_t i = lo + (uint32_t)j;
            int32_t K = offsets[i + 1] - offsets[i];
            if (ok[j])
                out[offsets[i] + K - 1] = rem[j];
            if (margin) margin[i] = mg[j];
        }
    }
}


void or_step_dirichlet(uint64_t seed, uint32_t unit0, uint32_t n_items, uint64_t *cursors,
                       const int32_t *offsets, const double *alpha, double *out,
                       double *tol, double *margin)
{
    int32_t kmax = 0;
    for (uint32_t i = 0; i < n_items; i++) {
        int32_t K = offsets[i + 1] - offsets[i];
        if (K > kmax)
            kmax = K;
    }
    double *y = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    double *yt = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
    for (uint32_t i = 0; i < n_items; i++) {
        stream_t s = {seed, unit0 + i, cursors + 4 * (size_t)i};
        int K = offsets[i + 1] - offsets[i];
        double m = dirichlet_item(&s, K, alpha + offsets[i], out + offsets[i],
                                  tol ? tol + offsets[i] : NULL, y, yt);
        if (margin)
            margin[i] = m;
    }
    free(y);
    free(yt);
}

/* One Dirichlet(alpha_0 .. alpha_{K-1}) whose gammas come from several units:
 * components [j tb, min(K, (j+1) tb)) are block j, drawn from unit unit0 + j
 * (cursors + 4 j) exactly as a K = tb item of that unit would draw them, and
 * theta_k = y_k / (sum of all K gammas).  A gamma's law does not depend on
 * which stream feeds it, so this is the same distribution as one item's
 * draw; with tb >= K it is that draw.  margin[j]: block j's smallest margin. */
void or_dirichlet_blocks(uint64_t seed, uint32_t unit0, int32_t K, int32_t tb, uint64_t *cursors,
                         const double *alpha, double *out, double *tol, double *margin)
{
    double *y = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    double *yt = (double *)malloc(sizeof(double) * (size_t)(K + 1));
    const int32_t nb = (K + tb - 1) / tb;
    for (int32_t j = 0; j < nb; j++) {
        const int32_t lo = j * tb, kb = (K - lo < tb) ? K - lo : tb;
        stream_t s = {seed, unit0 + (uint32_t)j, cursors + 4 * (size_t)j};
        const double m = gamma_comps(&s, kb, alpha + lo, y + lo, yt + lo);
        if (margin)
            margin[j] = m;
    }
    dirichlet_normalize(K, y, yt, out, tol);
    free(y);
    free(yt);
}

/* ------------------------------------------------------------------------ */
/* Multinomial(n, theta) from pool uniforms, integer exact.                 */
/*   q_k = rint(theta_k 2^24) (theta_k rounded to fp32 first: the integer   */
/*   decision is taken in the deviates' precision), Q = sum q_k (all q_k =  */
/*   1 if Q = 0), C_k = q_0 + ... + q_k.  Token i takes u_i from the U pool,*/
/*   j_i = (u_i 2^24 - 1)/2 in [0, 2^23), t_i = floor(j_i Q / 2^23), and    */
/*   falls in the first bin k with t_i < C_k.                               */
/* qdrift: allowed drift of each q_k (from theta's tolerance); the returned */
/* value is the smallest (distance of a t_i to a boundary) - (drift of that */
/* boundary); <= 0 means an implementation may place that token on the      */
/* other side.                                                              */
/* ------------------------------------------------------------------------ */

static double multinomial_item(stream_t *s, int K, int32_t ntok, const double *theta,
                               const double *ttol, int want_margin, int32_t *counts,
                               int64_t *C)
{
    int64_t Q = 0;
    for (int k = 0; k < K; k++) {
        float t32 = (float)theta[k];
        int64_t q = (int64_t)rint((double)t32 * 16777216.0);
        Q += q;
        C[k] = Q;
    }
    if (Q == 0) {
        for (int k = 0; k < K; k++)
            C[k] = k + 1;
        Q = K;
    }
    /* allowed drift of each boundary and of Q */
    double drift_acc = 0.0;
    double *drift = (double *)malloc(sizeof(double) * (size_t)K);
    for (int k = 0; k < K; k++) {
        drift_acc += 1.0 + (ttol ? ttol[k] : 0.0) * 16777216.0;
        drift[k] = drift_acc;
    }
    double dQ = drift_acc;
    double mmin = INFINITY;
    for (int k = 0; k < K; k++)
        counts[k] = 0;
    for (int32_t i = 0; i < ntok; i++) {
        double u = take(s, OR_U);
        int64_t j = (int64_t)((u * 16777216.0 - 1.0) / 2.0);
        int64_t t = (int64_t)(((uint64_t)j * (uint64_t)Q) >> 23);
        int bin = 0;
        while (!(t < C[bin]))
            bin++;
        counts[bin]++;
        if (!want_margin)
            continue;
        /* distance of t to every boundary, less that boundary's drift */
        for (int k = 0; k < K; k++) {
            double dist = fabs((double)t - (double)C[k]);
            double slack = dist - drift[k] - dQ - 1.0;
            if (slack < mmin)
                mmin = slack;
        }
    }
    free(drift);
    return mmin;
}

void or_multinomial(uint64_t seed, uint32_t unit0, uint32_t n_items, uint64_t *cursors,
                    const int32_t *offsets, const int32_t *ntok,
                    const double *theta, int32_t *counts)
{
    int32_t kmax = 1;
    for (uint32_t i = 0; i < n_items; i++)
        if (offsets[i + 1] - offsets[i] > kmax)
            kmax = offsets[i + 1] - offsets[i];
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)kmax);
    for (uint32_t i = 0; i < n_items; i++) {
        stream_t s = {seed, unit0 + i, cursors + 4 * (size_t)i};
        multinomial_item(&s, offsets[i + 1] - offsets[i], ntok[i],
                         theta + offsets[i], NULL, 0, counts + offsets[i], C);
    }
    free(C);
}

/* ------------------------------------------------------------------------ */
/* Chain models.  Traces are [step][slot]; slot p holds chain perm[p]       */
/* (identity when perm is NULL); units are `width` consecutive slots.       */
/* A chain c takes part in step t while t < steps[c].                       */
/* ------------------------------------------------------------------------ */

/* Triangle Gibbs sampler of Eq. 1 / Fig. 1, in double precision:
 * x <- U(0, 1 - y) then y <- U(0, 1 - x), starting from x = y = 0.5, both
 * from the U64 pool.  x0/y0 in, xf/yf out (user order). */
void or_triangle(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t iters,
                 const double *x0, const double *y0, uint64_t *cursors,
                 double *xtr, double *ytr, double *xf, double *yf)
{
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t s = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            xf[c] = x0 ? x0[c] : 0.5;
            yf[c] = y0 ? y0[c] : 0.5;
        }
        for (uint32_t t = 0; t < iters; t++) {
            for (uint32_t c = lo; c < hi; c++) { /* x call */
                double w = take(&s, OR_U64);
                xf[c] = 0.0 + (1.0 - yf[c] - 0.0) * w;
                if (xtr)
                    xtr[(size_t)t * n + c] = xf[c];
            }
            for (uint32_t c = lo; c < hi; c++) { /* y call */
                double w = take(&s, OR_U64);
                yf[c] = 0.0 + (1.0 - xf[c] - 0.0) * w;
                if (ytr)
                    ytr[(size_t)t * n + c] = yf[c];
            }
        }
    }
}

/* Varying-parameter normal/exponential chain:
 *   s_{t+1} ~ N(0.9 s_t, 0.5 + |s_t|), then e_{t+1} ~ Exp(1 + s_{t+1}^2).
 * fresh: s_0 is the chain's first Gaussian (one N call before step 0).
 * Traces str/etr [t][chain]; stol/etol carry first-order error bounds
 * propagated along the chain (local tolerance + |d s'/d s| times the
 * incoming bound). */
void or_normexp(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t steps,
                int fresh, double *s_state, uint64_t *cursors, double *str,
                double *etr, double *stol, double *etol)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    double *B = (double *)malloc(sizeof(double) * (size_t)(width));
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            if (fresh) {
                s_state[c] = take(&st, OR_N);
                B[c - lo] = or_tol(s_state[c]);
            } else {
                B[c - lo] = 0.0;
            }
        }
        for (uint32_t t = 0; t < steps; t++) {
            double sp[OR_MAXSLOT];
            for (uint32_t c = lo; c < hi; c++) { /* N call */
                double z = take(&st, OR_N);
                double s = s_state[c];
                double mu = 0.9 * s, sigma = 0.5 + fabs(s);
                sp[c - lo] = mu + sigma * z;
                double loc = or_tol(dmax(fabs(sp[c - lo]), dmax(fabs(mu), fabs(sigma * z))));
                double slope = fabs(0.9 + (s >= 0.0 ? z : -z));
                B[c - lo] = loc + slope * B[c - lo];
                str[(size_t)t * n + c] = sp[c - lo];
                if (stol)
                    stol[(size_t)t * n + c] = B[c - lo];
            }
            for (uint32_t c = lo; c < hi; c++) { /* E call */
                double e = take(&st, OR_E);
                double s = sp[c - lo];
                double lam = 1.0 + s * s;
                double v = e / lam;
                etr[(size_t)t * n + c] = v;
                if (etol)
                    etol[(size_t)t * n + c] =
                        or_tol(v) + fabs(2.0 * s * e / (lam * lam)) * B[c - lo];
                s_state[c] = s;
            }
        }
    }
    free(B);
}

/* Exponential chain (the served form's exponential kind):
 *   e_{t+1} ~ Exp(1 + e_t^2), i.e. E / (1 + e_t^2); fresh: e_0 is the
 * chain's first exponential.  Bounds propagate as in or_normexp. */
void or_expchain(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t steps,
                 int fresh, double *e_state, uint64_t *cursors, double *etr, double *etol)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    double B[OR_MAXSLOT];
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        for (uint32_t c = lo; c < hi; c++) {
            if (fresh) {
                e_state[c] = take(&st, OR_E);
                B[c - lo] = or_tol(e_state[c]);
            } else {
                B[c - lo] = 0.0;
            }
        }
        for (uint32_t t = 0; t < steps; t++) {
            for (uint32_t c = lo; c < hi; c++) {
                double E = take(&st, OR_E);
                double v = e_state[c];
                double lam = 1.0 + v * v;
                double nv = E / lam;
                B[c - lo] = or_tol(nv) + fabs(2.0 * v * E / (lam * lam)) * B[c - lo];
                e_state[c] = nv;
                etr[(size_t)t * n + c] = nv;
                if (etol)
                    etol[(size_t)t * n + c] = B[c - lo];
            }
        }
    }
}

/* Varying-shape gamma chain: alpha_{t+1} = 0.1 + g_t, g_t ~ Gamma(alpha_t, 1).
 * Each slot of a unit runs its own chain through the gamma rounds: when its
 * draw is accepted it starts the chain's next step in the next round.
 * alpha (user order) in: alpha_0, out: the next shape.  Slots follow perm,
 * steps[c] per chain.  gtr/gtol/gmar are [t][slot] (left untouched where a
 * chain has no step t); gr0/gr1 (may be null) receive each draw's start and
 * completion rounds, counted per unit from this call's first round. */
typedef struct {
    int L[OR_MAXSLOT], t[OR_MAXSLOT];
    double a[OR_MAXSLOT], ab[OR_MAXSLOT];
    uint32_t n, lo;
    double *gtr, *gtol, *gmar;
    int32_t *gr0, *gr1;
    const double *ash; /* replay: the shape of every draw, [t][slot], or NULL */
} chains_t;

static int chains_next(gsrc_t *g, int k, double *alpha, double *abound)
{
    chains_t *c = (chains_t *)g->ctx;
    if (c->t[k] >= c->L[k])
        return 0;
    *alpha = c->a[k];
    *abound = c->ab[k];
    return 1;
}

static void chains_done(gsrc_t *g, int k, const gdraw_t *r)
{
    chains_t *c = (chains_t *)g->ctx;
    size_t o = (size_t)c->t[k] * c->n + c->lo + (size_t)k;
    if (c->gtr) c->gtr[o] = r->g;
    if (c->gtol) c->gtol[o] = r->tol;
    if (c->gmar) c->gmar[o] = r->margin;
    if (c->gr0) c->gr0[o] = r->r0;
    if (c->gr1) c->gr1[o] = r->r1;
    c->t[k]++;
    if (c->ash) {
        /* replay: the next draw's shape is given exactly */
        if (c->t[k] < c->L[k])
            c->a[k] = c->ash[(size_t)c->t[k] * c->n + c->lo + (size_t)k];
        c->ab[k] = 0.0;
        return;
    }
    double an = 0.1 + r->g;
    /* the next shape carries g's bound plus the fp32 rounding of 0.1 + g
     * and of the constant 0.1 itself */
    c->ab[k] = r->tol + ulp32(an) + 2e-9;
    c->a[k] = an;
}

void or_gamma_chain(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, const int32_t *perm,
                    const int32_t *steps, double *alpha, uint64_t *cursors,
                    double *gtr, double *gtol, double *gmar, int32_t *gr0, int32_t *gr1)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    chains_t *cs = (chains_t *)malloc(sizeof(chains_t));
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        int ns = (int)(hi - lo);
        cs->n = n;
        cs->lo = lo;
        cs->gtr = gtr;
        cs->gtol = gtol;
        cs->gmar = gmar;
        cs->gr0 = gr0;
        cs->gr1 = gr1;
        cs->ash = NULL;
        for (int k = 0; k < ns; k++) {
            uint32_t ch = perm ? (uint32_t)perm[lo + k] : lo + k;
            cs->a[k] = alpha[ch];
            cs->ab[k] = 0.0;
            cs->t[k] = 0;
            cs->L[k] = steps[ch];
        }
        gsrc_t src = {chains_next, chains_done, cs};
        or_gamma_rounds(&st, ns, &src);
        for (int k = 0; k < ns; k++) {
            uint32_t ch = perm ? (uint32_t)perm[lo + k] : lo + k;
            alpha[ch] = cs->a[k];
        }
    }
    free(cs);
}

/* ------------------------------------------------------------------------ */
/* Per-step replay of the fp32 chain models.  A free-running chain in fp32  */
/* drifts away from its double-precision twin: each step amplifies the      */
/* rounding of the state it starts from.  Replay removes the drift from the */
/* check.  Every output is recomputed here from the state the implementation */
/* under test actually held before that step (given as input, exact), from  */
/* the same pool entries, in the same consumption order, so that each        */
/* output carries only its own step's rounding and is held to the single-   */
/* result bar max(4 ulp32(M), 1e-6 M).  The state values are inputs only:   */
/* nothing of the implementation's arithmetic enters the recomputation.     */
/* ------------------------------------------------------------------------ */

/* Normal/exponential chain, replayed.  s_in[t][chain] is the state before
 * step t (for t = 0 the starting state; for t > 0 the value the tested run
 * produced at step t - 1); sp_in[t][chain] is the s' of step t that the
 * tested run then used for its exponential.  fresh: the run first drew its
 * starting state as one N call, which is consumed here too (s0_ref receives
 * those Gaussians and s0_tol their bar; the replay itself starts from
 * s_in[0]).  Outputs as or_normexp, with local bars only. */
void or_normexp_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                       uint32_t steps, int fresh, const double *s_in, const double *sp_in,
                       uint64_t *cursors, double *s0_ref, double *s0_tol, double *str,
                       double *etr, double *stol, double *etol)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        if (fresh) {
            for (uint32_t c = lo; c < hi; c++) {
                double z0 = take(&st, OR_N);
                if (s0_ref) s0_ref[c] = z0;
                if (s0_tol) s0_tol[c] = or_tol(z0);
            }
        }
        for (uint32_t t = 0; t < steps; t++) {
            size_t row = (size_t)t * n;
            for (uint32_t c = lo; c < hi; c++) { /* N call */
                double z = take(&st, OR_N);
                double s = s_in[row + c];
                double mu = 0.9 * s, sigma = 0.5 + fabs(s);
                double sp = mu + sigma * z;
                str[row + c] = sp;
                stol[row + c] = or_tol(dmax(fabs(sp), dmax(fabs(mu), fabs(sigma * z))));
            }
            for (uint32_t c = lo; c < hi; c++) { /* E call */
                double e = take(&st, OR_E);
                double s = sp_in[row + c];
                double v = e / (1.0 + s * s);
                etr[row + c] = v;
                etol[row + c] = or_tol(v);
            }
        }
    }
}

/* Exponential chain, replayed: e_in[t][chain] is the state before step t
 * (as or_normexp_replay's s_in); fresh: the starting E call is consumed and
 * reported in e0_ref/e0_tol. */
void or_expchain_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                        uint32_t steps, int fresh, const double *e_in, uint64_t *cursors,
                        double *e0_ref, double *e0_tol, double *etr, double *etol)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        if (fresh) {
            for (uint32_t c = lo; c < hi; c++) {
                double e0 = take(&st, OR_E);
                if (e0_ref) e0_ref[c] = e0;
                if (e0_tol) e0_tol[c] = or_tol(e0);
            }
        }
        for (uint32_t t = 0; t < steps; t++) {
            size_t row = (size_t)t * n;
            for (uint32_t c = lo; c < hi; c++) {
                double E = take(&st, OR_E);
                double v = e_in[row + c];
                double nv = E / (1.0 + v * v);
                etr[row + c] = nv;
                etol[row + c] = or_tol(nv);
            }
        }
    }
}

/* Varying-shape gamma chain, replayed: shape[t][slot] is the shape of the
 * slot's draw at step t (for t = 0 the starting shape; for t > 0 what the
 * tested run formed from its own draw at step t - 1).  The slots run the
 * gamma rounds exactly as in or_gamma_chain, but every draw starts from its
 * given shape, which carries no error bound; outputs as or_gamma_chain. */
void or_gamma_chain_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                           const int32_t *perm, const int32_t *steps, const double *shape,
                           uint64_t *cursors, double *gtr, double *gtol, double *gmar,
                           int32_t *gr0, int32_t *gr1)
{
    if (width == 0 || width > OR_MAXSLOT)
        return;
    uint32_t nu = (n + width - 1) / width;
    chains_t *cs = (chains_t *)malloc(sizeof(chains_t));
    for (uint32_t u = 0; u < nu; u++) {
        stream_t st = {seed, unit0 + u, cursors + 4 * (size_t)u};
        uint32_t lo, hi;
        unit_range(n, width, u, &lo, &hi);
        int ns = (int)(hi - lo);
        cs->n = n;
        cs->lo = lo;
        cs->gtr = gtr;
        cs->gtol = gtol;
        cs->gmar = gmar;
        cs->gr0 = gr0;
        cs->gr1 = gr1;
        cs->ash = shape;
        for (int k = 0; k < ns; k++) {
            uint32_t ch = perm ? (uint32_t)perm[lo + k] : lo + k;
            cs->a[k] = shape[lo + (size_t)k];
            cs->ab[k] = 0.0;
            cs->t[k] = 0;
            cs->L[k] = steps[ch];
        }
        gsrc_t src = {chains_next, chains_done, cs};
        or_gamma_rounds(&st, ns, &src);
    }
    free(cs);
}

/* LDA-style Dirichlet resampling.  Unit = document d (key unit id d).
 * Per sweep: alpha_k = 0.1 + counts_k; theta ~ Dirichlet(alpha) (gamma
 * rounds over the components); counts ~ Multinomial(n_d, theta) with the
 * integer rule above.  counts (in/out) and the traces are laid out by the
 * component offsets; thtr/thtol/cntr are [sweep][total components],
 * gmar/mmar are [sweep][doc]. */
void or_lda(uint64_t seed, uint32_t unit0, uint32_t n_docs, const int32_t *offsets,
            const int32_t *ntok, uint32_t sweeps, int32_t *counts,
            uint64_t *cursors, double *thtr, double *thtol, int32_t *cntr,
            double *gmar, double *mmar)
{
    int32_t kmax = 1;
    for (uint32_t i = 0; i < n_docs; i++)
        if (offsets[i + 1] - offsets[i] > kmax)
            kmax = offsets[i + 1] - offsets[i];
    size_t total = (size_t)offsets[n_docs];
    double *al = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *th = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *tt = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *y = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *yt = (double *)malloc(sizeof(double) * (size_t)kmax);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)kmax);
    for (uint32_t d = 0; d < n_docs; d++) {
        stream_t st = {seed, unit0 + d, cursors + 4 * (size_t)d};
        int K = offsets[d + 1] - offsets[d];
        int32_t *cnt = counts + offsets[d];
        for (uint32_t sw = 0; sw < sweeps; sw++) {
            for (int k = 0; k < K; k++)
                al[k] = 0.1 + (double)cnt[k];
            double gm = dirichlet_item(&st, K, al, th, tt, y, yt);
            double mm = multinomial_item(&st, K, ntok[d], th, tt, mmar != NULL, cnt, C);
            for (int k = 0; k < K; k++) {
                size_t o = (size_t)sw * total + (size_t)offsets[d] + (size_t)k;
                if (thtr) thtr[o] = th[k];
                if (thtol) thtol[o] = tt[k];
                if (cntr) cntr[o] = cnt[k];
            }
            if (gmar) gmar[(size_t)sw * n_docs + d] = gm;
            if (mmar) mmar[(size_t)sw * n_docs + d] = mm;
        }
    }
    free(al); free(th); free(tt); free(y); free(yt); free(C);
}
