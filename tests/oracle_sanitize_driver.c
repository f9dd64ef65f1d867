/*
 * Drives every exported function of the CPU oracle (oracle/brng_oracle.c)
 * once on small, ragged inputs, with buffers allocated at their exact sizes,
 * so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * reports any out-of-bounds access or undefined operation.  Test
 * infrastructure only (tests/test_oracle_sanitizers.py builds and runs it);
 * it computes nothing of its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_philox4x32(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4]);
void or_block_words(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t block, uint32_t w[4]);
double or_u32(uint32_t w);
double or_u64(uint32_t wa, uint32_t wb);
double or_entry(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t j);
void or_entries(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t j0, uint64_t n, double *out);
void or_convert(int kind, const uint32_t *w, uint64_t n_words, double *out);
void or_u32_many(const uint32_t *w, uint64_t n, double *out);
void or_words(uint64_t seed, uint32_t unit, uint32_t kind, uint64_t b0, uint64_t nb, uint32_t *out);
double or_tol(double m);
void or_step_uniform(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, int kind,
                     uint64_t *cursors, const double *a, const double *b, double *out, double *tol);
void or_step_normal(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                    const double *mu, const double *sigma, double *out, double *tol);
void or_step_exp(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                 const double *lambda, double *out, double *tol);
void or_step_laplace(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *mu, const double *b, double *out, double *tol);
void or_step_weibull(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *lambda, const double *k, double *out, double *tol);
void or_step_gamma(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                   const double *alpha, double *out, double *tol, double *margin, int32_t *nN,
                   int32_t *nE);
void or_step_poisson(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint64_t *cursors,
                     const double *lambda, int32_t *out, double *margin);
void or_step_binomial(uint64_t seed, uint32_t unit0, uint32_t n_ch, uint32_t width,
                      uint64_t *cursors, const int32_t *nn, const double *pr, int32_t *out,
                      double *margin);
void or_step_multinomial(uint64_t seed, uint32_t unit0, uint32_t n_items, uint32_t width,
                         uint64_t *cursors, const int32_t *offsets, const int32_t *nn,
                         const double *pw, int32_t *out, double *margin);
void or_step_dirichlet(uint64_t seed, uint32_t unit0, uint32_t n_items, uint64_t *cursors,
                       const int32_t *offsets, const double *alpha, double *out, double *tol,
                       double *margin);
void or_multinomial(uint64_t seed, uint32_t unit0, uint32_t n_items, uint64_t *cursors,
                    const int32_t *offsets, const int32_t *ntok, const double *theta,
                    int32_t *counts);
void or_triangle(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t iters,
                 const double *x0, const double *y0, uint64_t *cursors, double *xtr, double *ytr,
                 double *xf, double *yf);
void or_normexp(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t steps,
                int fresh, double *s_state, uint64_t *cursors, double *str, double *etr,
                double *stol, double *etol);
void or_expchain(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t steps,
                 int fresh, double *e_state, uint64_t *cursors, double *etr, double *etol);
void or_gamma_chain(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                    const int32_t *perm, const int32_t *steps, double *alpha, uint64_t *cursors,
                    double *gtr, double *gtol, double *gmar, int32_t *gr0, int32_t *gr1);
void or_normexp_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width, uint32_t steps,
                       int fresh, const double *s_in, const double *sp_in, uint64_t *cursors,
                       double *s0_ref, double *s0_tol, double *str, double *etr, double *stol,
                       double *etol);
void or_expchain_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                        uint32_t steps, int fresh, const double *e_in, uint64_t *cursors,
                        double *e0_ref, double *e0_tol, double *etr, double *etol);
void or_gamma_chain_replay(uint64_t seed, uint32_t unit0, uint32_t n, uint32_t width,
                           const int32_t *perm, const int32_t *steps, const double *shape,
                           uint64_t *cursors, double *gtr, double *gtol, double *gmar,
                           int32_t *gr0, int32_t *gr1);
void or_lda(uint64_t seed, uint32_t unit0, uint32_t n_docs, const int32_t *offsets,
            const int32_t *ntok, uint32_t sweeps, int32_t *counts, uint64_t *cursors,
            double *thtr, double *thtol, int32_t *cntr, double *gmar, double *mmar);

#define NEW(T, n) ((T *)calloc((size_t)(n), sizeof(T)))

static uint64_t *cursors(uint32_t units) { return NEW(uint64_t, 4 * (size_t)units); }

static double lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * 0x1p-53;
}

int main(void)
{
    uint64_t rs = 7;
    /* engine and conversions */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w4[4];
    or_philox4x32(ctr, key, 10, w4);
    or_block_words(0xFFFFFFFF00000005ull, 3, 2, (1ull << 34) + 1, w4);
    volatile double sink = or_u32(0) + or_u32(0xFFFFFFFFu) + or_u64(0, 0) + or_u64(~0u, ~0u);
    sink += or_entry(1, 2, 3, 5) + or_tol(0.0) + or_tol(1e-40) + or_tol(3e38);
    for (int kind = 0; kind < 4; kind++) {
        double *e = NEW(double, 37);
        or_entries(9, 1, (uint32_t)kind, 3, 37, e);
        free(e);
        uint32_t *w = NEW(uint32_t, 12);
        or_words(9, 1, (uint32_t)kind, 0, 3, w);
        double *c = NEW(double, 12);
        or_convert(kind, w, 12, c);
        or_u32_many(w, 12, c);
        free(c);
        free(w);
    }
    /* step calls: a partial second unit (n = 100, width 64) */
    const uint32_t n = 100, nu = 2;
    double *a = NEW(double, n), *b = NEW(double, n), *out = NEW(double, n), *tol = NEW(double, n);
    double *mar = NEW(double, n);
    int32_t *i1 = NEW(int32_t, n), *i2 = NEW(int32_t, n), *io = NEW(int32_t, n);
    for (uint32_t i = 0; i < n; i++) {
        a[i] = lcg(&rs) * 4.0 - 2.0;
        b[i] = a[i] + 0.5 + lcg(&rs);
    }
    uint64_t *cur = cursors(nu);
    or_step_uniform(3, 0, n, 64, 0, cur, a, b, out, tol);
    or_step_uniform(3, 0, n, 64, 3, cur, a, b, out, tol);
    or_step_normal(3, 0, n, 64, cur, a, b, out, tol);
    or_step_exp(3, 0, n, 64, cur, b, out, tol);
    or_step_laplace(3, 0, n, 64, cur, a, b, out, tol);
    or_step_weibull(3, 0, n, 64, cur, b, b, out, tol);
    for (uint32_t i = 0; i < n; i++)
        a[i] = exp(lcg(&rs) * 12.0 - 4.0); /* shapes 0.018..2980 */
    a[3] = 0.0;                            /* invalid shape */
    a[4] = NAN;
    or_step_gamma(3, 0, n, 64, cur, a, out, tol, mar, i1, i2);
    for (uint32_t i = 0; i < n; i++) {
        a[i] = exp(lcg(&rs) * 14.0 - 5.0); /* rates 0.007..8000 */
        i1[i] = (int32_t)(lcg(&rs) * 5000.0);
        b[i] = lcg(&rs);
    }
    a[0] = -1.0;
    i1[1] = -3;
    b[2] = 1.5;
    or_step_poisson(3, 0, n, 64, cur, a, io, mar);
    or_step_binomial(3, 0, n, 64, cur, i1, b, io, mar);
    free(cur);
    /* ragged items: multinomial and Dirichlet, K from 0 to 300 */
    const uint32_t ni = 6;
    int32_t off[7] = {0, 1, 5, 5, 69, 200, 500};
    int32_t tot = off[ni];
    double *w = NEW(double, tot), *dout = NEW(double, tot), *dtol = NEW(double, tot);
    int32_t *cnt = NEW(int32_t, tot), nn[6] = {3, 100, 5, 1000, 0, 257};
    for (int32_t i = 0; i < tot; i++)
        w[i] = 0.05 + lcg(&rs) * 3.0;
    cur = cursors(ni);
    or_step_multinomial(5, 0, ni, 64, cur, off, nn, w, cnt, mar);
    double *imar = NEW(double, ni);
    int32_t offd[6] = {0, 1, 5, 69, 200, 500};
    or_step_dirichlet(5, 0, 5, cur, offd, w, dout, dtol, imar);
    or_multinomial(5, 0, 5, cur, offd, nn, dout, cnt);
    free(cur);
    /* chain models */
    const uint32_t nc = 70, steps = 9;
    double *x0 = NEW(double, nc), *y0 = NEW(double, nc), *xf = NEW(double, nc), *yf = NEW(double, nc);
    double *tr1 = NEW(double, (size_t)steps * nc), *tr2 = NEW(double, (size_t)steps * nc);
    double *tr3 = NEW(double, (size_t)steps * nc), *tr4 = NEW(double, (size_t)steps * nc);
    for (uint32_t i = 0; i < nc; i++) x0[i] = y0[i] = 0.25;
    cur = cursors(2);
    or_triangle(1, 0, nc, 64, steps, x0, y0, cur, tr1, tr2, xf, yf);
    or_triangle(1, 0, nc, 64, steps, NULL, NULL, cur, NULL, NULL, xf, yf);
    double *s = NEW(double, nc), *s0r = NEW(double, nc), *s0t = NEW(double, nc);
    or_normexp(1, 0, nc, 64, steps, 1, s, cur, tr1, tr2, tr3, tr4);
    or_normexp(1, 0, nc, 64, steps, 0, s, cur, tr1, tr2, NULL, NULL);
    or_normexp_replay(1, 0, nc, 64, steps, 1, tr1, tr1, cur, s0r, s0t, tr2, tr3, tr4, tr2);
    or_expchain(1, 0, nc, 64, steps, 1, s, cur, tr1, tr2);
    or_expchain_replay(1, 0, nc, 64, steps, 1, tr1, cur, s0r, s0t, tr2, tr3);
    int32_t *perm = NEW(int32_t, nc), *st = NEW(int32_t, nc);
    int32_t *g0 = NEW(int32_t, (size_t)steps * nc), *g1 = NEW(int32_t, (size_t)steps * nc);
    for (uint32_t i = 0; i < nc; i++) {
        perm[i] = (int32_t)(nc - 1 - i);
        st[i] = 1 + (int32_t)(i % steps);
        s[i] = exp(lcg(&rs) * 6.0 - 2.3);
    }
    or_gamma_chain(1, 0, nc, 64, perm, st, s, cur, tr1, tr2, tr3, g0, g1);
    for (size_t i = 0; i < (size_t)steps * nc; i++)
        tr4[i] = 0.5 + lcg(&rs) * 3.0;
    or_gamma_chain_replay(1, 0, nc, 64, perm, st, tr4, cur, tr1, tr2, tr3, g0, g1);
    free(cur);
    /* LDA-style documents, K = 1, 4, 64, 131, 300 */
    const uint32_t nd = 5, sw = 3;
    int32_t loff[6] = {0, 1, 5, 69, 200, 500}, ntk[5] = {0, 7, 200, 64, 129};
    int32_t *lc = NEW(int32_t, 500), *lct = NEW(int32_t, (size_t)sw * 500);
    double *lth = NEW(double, (size_t)sw * 500), *ltt = NEW(double, (size_t)sw * 500);
    double *lgm = NEW(double, (size_t)sw * nd), *lmm = NEW(double, (size_t)sw * nd);
    cur = cursors(nd);
    or_lda(2, 0, nd, loff, ntk, sw, lc, cur, lth, ltt, lct, lgm, lmm);
    or_lda(2, 0, nd, loff, ntk, sw, lc, cur, NULL, NULL, NULL, NULL, NULL);
    free(cur);
    printf("driver ok %d\n", sink != 12345.0);
    free(a); free(b); free(out); free(tol); free(mar); free(i1); free(i2); free(io);
    free(w); free(dout); free(dtol); free(cnt); free(imar);
    free(x0); free(y0); free(xf); free(yf); free(tr1); free(tr2); free(tr3); free(tr4);
    free(s); free(s0r); free(s0t); free(perm); free(st); free(g0); free(g1);
    free(lc); free(lct); free(lth); free(ltt); free(lgm); free(lmm);
    return 0;
}
