/*
 * Differential evolution per domain and the evolution-by-neighbourhood-
 * similarity (ENS) sweep.  Test infrastructure (see oracle.h).
 *
 * Per domain (ZO sample), section "JADE applied to traveltime parameter
 * search": NP individuals drawn uniformly in the parameter box and scored
 * (Initializing); the best individual located (Sorting, with P = 1 so the
 * p-best is the best); for each individual i a mutant built from i, the best
 * and two other random members (Mutation and crossover, current-to-best/1),
 * crossed with i; all trials scored, then each trial replaces its parent when
 * its semblance is at least as large, the old population being kept until
 * every comparison is made (Selection).  After NG generations the best is
 * returned.  Evaluations per domain: NP (1 + NG) (eq. jade_semblance).
 *
 * Control parameters.  The paper runs JADE with archive in every domain and
 * takes its adaptation from earlier work without stating it (sections
 * "Selection", "Evolution by neighborhood similarity").  adapt = 0: constant
 * F and CR.  adapt = 1: JADE (Zhang and Sanderson, 2009) with P = 1:
 *   - per generation and slot, CR_i ~ N(mu_CR, 0.1) clipped to [0, 1] and
 *     F_i ~ Cauchy(mu_F, 0.1), 1 where above 1, redrawn where not positive
 *     (three draws, then mu_F); both are kept on the grid k / 2^24 so that
 *     their sums below are exact integers;
 *   - the second difference vector's minuend x_r2 comes from the population
 *     joined with the archive A of replaced parents (|A| <= NP);
 *   - every replaced parent enters A (appended while |A| < NP, else
 *     overwriting a uniformly drawn position), in slot order;
 *   - after the generation, when some trial replaced its parent,
 *     mu_CR <- 0.9 mu_CR + 0.1 mean(CR of those slots) and
 *     mu_F <- 0.9 mu_F + 0.1 sum F^2 / sum F over them (Lehmer mean);
 *   - each domain (sample and stage) starts from mu_CR = CR, mu_F = F and an
 *     empty archive.
 * Binomial crossover has one forced dimension, and out-of-box mutant
 * coordinates are repaired to the midpoint between bound and parent.
 *
 * Random numbers: one Philox-4x64-10 block per (sample, stage, generation,
 * slot), key (seed, 0).  Generation 0 words 0..2 give the initial coordinates
 * (top 24 bits as a binary32 fraction); later generations: word 0 high/low
 * halves draw r1 in [0,NP-1) and r2 in [0,NP-2) by multiply-shift, skipping
 * the excluded indices in ascending order; word 1 high half draws the forced
 * dimension; word 1 low, word 2 high, word 2 low are the crossover draws of
 * dimensions 0, 1, 2, compared against ceil(CR 2^32).  With the archive, r2
 * is drawn in [0, NP + |A| - 2) the same way (indices from NP on name
 * archive entries).  JADE's draws come from a second block per (sample,
 * generation, slot), stage word + 2^32: words 0 and 1 (top 53 bits) give the
 * Box-Muller normal for CR, the halves of word 2 and the high half of word 3
 * the Cauchy draws for F (inverse CDF), the low half of word 3 the archive
 * position.
 *
 * ENS (sections "Information propagation" and "Evolution by neighborhood
 * similarity"), first with N_skip = 0: stage 0 sweeps each interactive domain (bucket of
 * consecutive output CMPs) left to right with NP_f, NG_f; the best of
 * (t, previous trace) replaces slot 0 of (t, trace).  Each of the N_cycle
 * cycles then sweeps right to left and left to right with NP_bf, NG_bf; slots
 * 0, 1, 2 take the bests of (t-1, trace), (t+1, trace) and (t, previous trace
 * of this sweep), slot 3 the current best of (t, trace) with its stored
 * score (not re-evaluated), the rest are random; a missing neighbour leaves
 * its slot random.  All t of one trace step read the state as it was before
 * the step (the t are processed concurrently).  Evaluations per sample:
 * NP_f (1 + NG_f) + N_cycle 2 (NP_bf (1 + NG_bf) - 1) (eq. ens_semblance).
 *
 * Time-sample skipping (section "The performance-quality trade-off by an
 * interpolation process" and the stage definitions of section "Evolution by
 * neighborhood similarity"), N_skip in {1, 2}: each stage estimates only the
 * samples t = t_begin + init + m (N_skip + 1), with init 0 for the first
 * forward sweep, min(1, N_skip) for backward sweeps and N_skip for the later
 * forward sweeps.  After a trace's estimation the other samples of that
 * trace take the parameters interpolated linearly in t between the nearest
 * estimated samples of this stage on either side (the nearest one alone at
 * the ends of the grid), clamped into their own box, and are scored once.
 * In the first stage that is their result; in later stages the interpolated
 * individual replaces the stored one only when it scores higher.  Each
 * skipped sample costs one evaluation per stage (eq. ens_semblance).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

#define MAXNP 64

int32_t or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t or_pop_size(const or_de_cfg *cfg, int32_t nt, int32_t n0)
{
    if (nt <= 1)
        return cfg->np_lo;
    double v = cfg->np_lo + (double)(cfg->np_hi - cfg->np_lo) * (double)n0 / (double)(nt - 1);
    return (int32_t)floor(v + 0.5);
}

void or_sample_bounds(const or_line *L, const or_bounds *B, int32_t n0, float lo[3], float hi[3])
{
    const float dt = (float)L->dt;
    const float t0 = (float)n0 * dt;
    const float den = t0 > dt ? t0 : dt;
    for (int d = 0; d < 3; ++d) {
        lo[d] = B->lo[d];
        hi[d] = B->hi[d];
        if (B->inv_t0_mask >> d & 1u) {
            lo[d] = lo[d] / den;
            hi[d] = hi[d] / den;
        }
    }
}

static void rng_words(uint64_t seed, uint64_t sample, uint64_t stage, uint64_t gen, uint64_t slot,
                      uint64_t w[4])
{
    const uint64_t ctr[4] = {sample, stage, gen, slot};
    const uint64_t key[2] = {seed, 0};
    or_philox4x64_10(ctr, key, w);
}

static void random_individual(const uint64_t w[4], int P, const float *lo, const float *hi,
                              float *x)
{
    for (int d = 0; d < P; ++d) {
        float u = (float)(w[d] >> 40) * 0x1p-24f;
        float range = hi[d] - lo[d];
        float step = u * range;
        x[d] = lo[d] + step;
    }
}

void or_de_trial(int32_t np, int32_t P, const float *pop, const double *S, const uint64_t *words,
                 float F, float CR, const float *lo, const float *hi, float *trial)
{
    int32_t b = 0;
    for (int32_t i = 1; i < np; ++i)
        if (S[i] > S[b])
            b = i;
    const uint64_t thr = (uint64_t)ceil((double)CR * 4294967296.0);
    for (int32_t i = 0; i < np; ++i) {
        const uint64_t *w = words + 4 * i;
        uint32_t r1 = (uint32_t)(((w[0] >> 32) * (uint64_t)(np - 1)) >> 32);
        if (r1 >= (uint32_t)i)
            r1 += 1;
        uint32_t r2 = (uint32_t)(((w[0] & 0xffffffffULL) * (uint64_t)(np - 2)) >> 32);
        uint32_t ex_lo = (uint32_t)i < r1 ? (uint32_t)i : r1;
        uint32_t ex_hi = (uint32_t)i < r1 ? r1 : (uint32_t)i;
        if (r2 >= ex_lo)
            r2 += 1;
        if (r2 >= ex_hi)
            r2 += 1;
        uint32_t jr = (uint32_t)(((w[1] >> 32) * (uint64_t)P) >> 32);
        uint64_t cr[3] = {w[1] & 0xffffffffULL, w[2] >> 32, w[2] & 0xffffffffULL};
        for (int d = 0; d < P; ++d) {
            float xi = pop[i * P + d];
            float t1 = pop[b * P + d] - xi;
            float t2 = pop[r1 * P + d] - pop[r2 * P + d];
            float m1 = F * t1;
            float m2 = F * t2;
            float v = xi + m1;
            v = v + m2;
            if (v < lo[d])
                v = (lo[d] + xi) * 0.5f;
            else if (v > hi[d])
                v = (hi[d] + xi) * 0.5f;
            int take = (cr[d] < thr) || ((uint32_t)d == jr);
            trial[i * P + d] = take ? v : xi;
        }
    }
}

#define JADE_GRID 16777216.0 /* 2^24 */
#define PI_D 3.14159265358979323846
#define LN2_D 0.693147180559945309417

/* The variates use their own binary64 series (no library transcendental),
 * each operation written out, so that any IEEE binary64 implementation of
 * + - * / and sqrt produces the same bits:
 *   ln u = e ln 2 + 2 atanh((m-1)/(m+1)), u = m 2^e, m in [sqrt(1/2), sqrt(2)),
 *          atanh by its Taylor series to the s^23 term (|s| <= 0.172);
 *   sin a, cos a for a in [0, pi/2] by their Taylor series to a^25, a^24. */
static double jade_ln(double u)
{
    int e;
    double m = frexp(u, &e);
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = 1.0 / 23.0;
    for (int k = 21; k >= 1; k -= 2)
        p = p * s2 + 1.0 / (double)k;
    return (double)e * LN2_D + 2.0 * s * p;
}

static void jade_sincos(double a, double *sn, double *cs)
{
    const double a2 = a * a;
    double ps = 1.0, pc = 1.0;
    /* Horner from the highest term: sin a = a (1 - a^2/(2 3) (1 - a^2/(4 5) (...))) */
    for (int k = 24; k >= 2; k -= 2) {
        ps = 1.0 - ps * a2 / (double)((k) * (k + 1));
        pc = 1.0 - pc * a2 / (double)((k - 1) * (k));
    }
    *sn = a * ps;
    *cs = pc;
}

/* cos(2 pi t), t in [0, 1): quarter turn q and the angle within it */
static double jade_cos_turns(double t)
{
    const double v = 4.0 * t;
    const double q = floor(v);
    const double a = (v - q) * (PI_D / 2.0);
    double sn, cs;
    jade_sincos(a, &sn, &cs);
    const int iq = (int)q;
    return iq == 0 ? cs : (iq == 1 ? -sn : (iq == 2 ? -cs : sn));
}

/* tan(pi x), x in (-1/2, 1/2) */
static double jade_tan_half_turn(double x)
{
    const double y = x < 0.0 ? -x : x;
    double sn, cs;
    jade_sincos(y * PI_D, &sn, &cs);
    const double t = sn / cs;
    return x < 0.0 ? -t : t;
}

double or_jade_ln(double u) { return jade_ln(u); }
double or_jade_cos_turns(double t) { return jade_cos_turns(t); }
double or_jade_tan_half_turn(double x) { return jade_tan_half_turn(x); }

void or_jade_series_batch(int32_t which, int64_t n, const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = which == 0 ? jade_ln(x[i]) : (which == 1 ? jade_cos_turns(x[i]) : jade_tan_half_turn(x[i]));
}

void or_jade_draws(const uint64_t w[4], double mu_cr, double mu_f, int32_t np, int32_t *k_cr,
                   int32_t *k_f, int32_t *a_idx)
{
    /* CR: Box-Muller normal from two 53-bit uniforms, u1 in (0, 1] */
    const double u1 = ((double)(w[0] >> 11) + 1.0) * 0x1p-53;
    const double u2 = (double)(w[1] >> 11) * 0x1p-53;
    const double z = sqrt(-2.0 * jade_ln(u1)) * jade_cos_turns(u2);
    double cr = mu_cr + 0.1 * z;
    if (cr < 0.0)
        cr = 0.0;
    if (cr > 1.0)
        cr = 1.0;
    *k_cr = (int32_t)nearbyint(cr * JADE_GRID);
    /* F: Cauchy by the inverse CDF from 32-bit uniforms in (0, 1) */
    const uint64_t h[3] = {w[2] >> 32, w[2] & 0xffffffffULL, w[3] >> 32};
    int32_t kf = 0;
    for (int a = 0; a < 3 && kf == 0; ++a) {
        const double u = ((double)h[a] + 0.5) * 0x1p-32;
        double f = mu_f + 0.1 * jade_tan_half_turn(u - 0.5);
        if (f > 1.0)
            f = 1.0;
        if (f > 0.0)
            kf = (int32_t)nearbyint(f * JADE_GRID);
    }
    if (kf == 0) {
        kf = (int32_t)nearbyint(mu_f * JADE_GRID);
        if (kf < 1)
            kf = 1;
    }
    *k_f = kf;
    *a_idx = (int32_t)(((w[3] & 0xffffffffULL) * (uint64_t)np) >> 32);
}

void or_jade_trial(int32_t np, int32_t P, const float *pop, const double *S, const float *archive,
                   int32_t n_arch, const uint64_t *words, const int32_t *k_f, const int32_t *k_cr,
                   const float *lo, const float *hi, float *trial)
{
    int32_t b = 0;
    for (int32_t i = 1; i < np; ++i)
        if (S[i] > S[b])
            b = i;
    const int32_t total = np + n_arch;
    for (int32_t i = 0; i < np; ++i) {
        const uint64_t *w = words + 4 * i;
        uint32_t r1 = (uint32_t)(((w[0] >> 32) * (uint64_t)(np - 1)) >> 32);
        if (r1 >= (uint32_t)i)
            r1 += 1;
        uint32_t r2 = (uint32_t)(((w[0] & 0xffffffffULL) * (uint64_t)(total - 2)) >> 32);
        uint32_t ex_lo = (uint32_t)i < r1 ? (uint32_t)i : r1;
        uint32_t ex_hi = (uint32_t)i < r1 ? r1 : (uint32_t)i;
        if (r2 >= ex_lo)
            r2 += 1;
        if (r2 >= ex_hi)
            r2 += 1;
        const float *x2 = r2 < (uint32_t)np ? pop + r2 * P : archive + (r2 - (uint32_t)np) * P;
        uint32_t jr = (uint32_t)(((w[1] >> 32) * (uint64_t)P) >> 32);
        uint64_t cr[3] = {w[1] & 0xffffffffULL, w[2] >> 32, w[2] & 0xffffffffULL};
        const uint64_t thr = (uint64_t)k_cr[i] << 8; /* CR 2^32, exact on the grid */
        const float F = (float)k_f[i] * 0x1p-24f;
        for (int d = 0; d < P; ++d) {
            float xi = pop[i * P + d];
            float t1 = pop[b * P + d] - xi;
            float t2 = pop[r1 * P + d] - x2[d];
            float m1 = F * t1;
            float m2 = F * t2;
            float v = xi + m1;
            v = v + m2;
            if (v < lo[d])
                v = (lo[d] + xi) * 0.5f;
            else if (v > hi[d])
                v = (hi[d] + xi) * 0.5f;
            int take = (cr[d] < thr) || ((uint32_t)d == jr);
            trial[i * P + d] = take ? v : xi;
        }
    }
}

/* ---------------------------------------------------------------------------
 * objective */

typedef struct {
    const or_line *L;
    const or_de_cfg *cfg;
    int P;
} objective_ctx;

static double objective(const objective_ctx *o, int32_t j, int32_t n0, const float *x,
                        const float *lo, const float *hi)
{
    if (o->cfg->objective == 0) {
        double p[3] = {0, 0, 0};
        for (int d = 0; d < o->P; ++d)
            p[d] = (double)x[d];
        return or_semblance(o->L, j, n0, p, NULL, NULL);
    }
    /* mock objectives in box-normalised coordinates, optimum at c_d = 0.3 + 0.1 d */
    double r2 = 0.0, inside = 1.0;
    for (int d = 0; d < o->P; ++d) {
        double z = ((double)x[d] - lo[d]) / ((double)hi[d] - lo[d]);
        double c = 0.3 + 0.1 * d;
        r2 += (z - c) * (z - c);
        if (fabs(z - c) > 0.02)
            inside = 0.0;
    }
    if (o->cfg->objective == 1)
        return 1.0 / (1.0 + 50.0 * r2);
    return inside;
}

/* JADE's state of one domain: the control-parameter means and the archive
 * of replaced parents. */
typedef struct {
    double mu_cr, mu_f;
    int32_t n_arch;
    float archive[MAXNP * 3];
} jade_state;

/* Synchronous selection after a generation's trials are scored (section
 * "Selection"): trial i replaces parent i when St[i] >= S[i].  With JADE's
 * adaptation, in slot order every replaced parent enters the archive
 * (appended while it holds fewer than np entries, else at that slot's drawn
 * position a_idx[i]) and the slot's CR and F join the successful sets; then,
 * if any slot succeeded, mu_CR moves 10% toward the arithmetic mean of the
 * successful CR and mu_F 10% toward the Lehmer mean (sum F^2 / sum F) of the
 * successful F.  CR and F are k / 2^24, so the sums are exact integers. */
static void select_and_adapt(int np, int P, int adapt, const float *trial, const double *St, float *pop,
                             double *S, const int32_t *k_cr, const int32_t *k_f, const int32_t *a_idx,
                             jade_state *js)
{
    int64_t n_succ = 0, sum_cr = 0, sum_f = 0, sum_f2 = 0;
    for (int i = 0; i < np; ++i) {
        if (St[i] >= S[i]) {
            if (adapt) {
                float *dst = js->n_arch < np ? js->archive + (js->n_arch++) * P : js->archive + a_idx[i] * P;
                memcpy(dst, pop + i * P, sizeof(float) * (size_t)P);
                n_succ += 1;
                sum_cr += k_cr[i];
                sum_f += k_f[i];
                sum_f2 += (int64_t)k_f[i] * k_f[i];
            }
            memcpy(pop + i * P, trial + i * P, sizeof(float) * (size_t)P);
            S[i] = St[i];
        }
    }
    if (adapt && n_succ > 0) {
        const double mean_cr = (double)sum_cr / ((double)n_succ * JADE_GRID);
        const double lehmer_f = (double)sum_f2 / ((double)sum_f * JADE_GRID);
        js->mu_cr = 0.9 * js->mu_cr + 0.1 * mean_cr;
        js->mu_f = 0.9 * js->mu_f + 0.1 * lehmer_f;
    }
}

/* Trial vectors of one generation: fixed F and CR, or JADE's per-slot draws
 * (from the slots' adaptation blocks jw at the current means) with the
 * archive feeding x_r2. */
static void make_trials(int np, int P, int adapt, float F, float CR, const float *pop, const double *S,
                        const uint64_t *words, const uint64_t *jw, const float *lo, const float *hi,
                        jade_state *js, int32_t *k_cr, int32_t *k_f, int32_t *a_idx, float *trial)
{
    if (adapt) {
        for (int i = 0; i < np; ++i)
            or_jade_draws(jw + 4 * i, js->mu_cr, js->mu_f, np, &k_cr[i], &k_f[i], &a_idx[i]);
        or_jade_trial(np, P, pop, S, js->archive, js->n_arch, words, k_f, k_cr, lo, hi, trial);
    } else {
        or_de_trial(np, P, pop, S, words, F, CR, lo, hi, trial);
    }
}

/* NG generations of DE on one domain; pop/S hold the scored initial
 * population on entry and the final one on exit.  Returns evaluations. */
static int64_t evolve(const objective_ctx *o, uint64_t seed, uint64_t sample, uint64_t stage,
                      int32_t j, int32_t n0, int np, int ng, const float *lo, const float *hi,
                      float *pop, double *S)
{
    const int P = o->P;
    float trial[MAXNP * 3];
    double St[MAXNP];
    uint64_t words[MAXNP * 4], jw[MAXNP * 4];
    int64_t evals = 0;
    const int adapt = o->cfg->adapt;
    jade_state js;
    js.mu_cr = (double)o->cfg->CR;
    js.mu_f = (double)o->cfg->F;
    js.n_arch = 0;
    int32_t k_cr[MAXNP], k_f[MAXNP], a_idx[MAXNP];
    for (int g = 1; g <= ng; ++g) {
        for (int i = 0; i < np; ++i) {
            rng_words(seed, sample, stage, (uint64_t)g, (uint64_t)i, words + 4 * i);
            if (adapt)
                rng_words(seed, sample, stage + (1ULL << 32), (uint64_t)g, (uint64_t)i, jw + 4 * i);
        }
        make_trials(np, P, adapt, o->cfg->F, o->cfg->CR, pop, S, words, jw, lo, hi, &js, k_cr, k_f, a_idx,
                    trial);
        for (int i = 0; i < np; ++i) {
            St[i] = objective(o, j, n0, trial + i * P, lo, hi);
            ++evals;
        }
        select_and_adapt(np, P, adapt, trial, St, pop, S, k_cr, k_f, a_idx, &js);
    }
    return evals;
}

void or_jade_run(int32_t np, int32_t P, float *pop, double *S, int32_t ng, const uint64_t *de_words,
                 const uint64_t *jade_words, const int32_t *draws, const double *St, float F0, float CR0,
                 const float *lo, const float *hi, float *trials_out, double *mu_out, int32_t *n_arch_out,
                 float *archive_out)
{
    jade_state js;
    js.mu_cr = (double)CR0;
    js.mu_f = (double)F0;
    js.n_arch = 0;
    memset(js.archive, 0, sizeof js.archive);
    int32_t k_cr[MAXNP], k_f[MAXNP], a_idx[MAXNP];
    for (int32_t g = 0; g < ng; ++g) {
        const uint64_t *w = de_words + (size_t)g * np * 4;
        if (jade_words) {
            make_trials(np, P, 1, F0, CR0, pop, S, w, jade_words + (size_t)g * np * 4, lo, hi, &js, k_cr, k_f,
                        a_idx, trials_out + (size_t)g * np * P);
        } else {
            for (int32_t i = 0; i < np; ++i) {
                const int32_t *d = draws + ((size_t)g * np + i) * 3;
                k_cr[i] = d[0];
                k_f[i] = d[1];
                a_idx[i] = d[2];
            }
            or_jade_trial(np, P, pop, S, js.archive, js.n_arch, w, k_f, k_cr, lo, hi,
                          trials_out + (size_t)g * np * P);
        }
        select_and_adapt(np, P, 1, trials_out + (size_t)g * np * P, St + (size_t)g * np, pop, S, k_cr, k_f,
                         a_idx, &js);
        mu_out[2 * g] = js.mu_cr;
        mu_out[2 * g + 1] = js.mu_f;
        n_arch_out[g] = js.n_arch;
        memcpy(archive_out + (size_t)g * np * P, js.archive, sizeof(float) * (size_t)np * P);
    }
}

static int best_index(const double *S, int np)
{
    int b = 0;
    for (int i = 1; i < np; ++i)
        if (S[i] > S[b])
            b = i;
    return b;
}

static void clamp_into(float *x, int P, const float *lo, const float *hi)
{
    for (int d = 0; d < P; ++d) {
        if (x[d] < lo[d])
            x[d] = lo[d];
        if (x[d] > hi[d])
            x[d] = hi[d];
    }
}

static int64_t plain_de(const objective_ctx *o, const or_bounds *B, uint64_t seed,
                        const int32_t *cmp_out, int32_t n_out, int32_t t_begin, int32_t t_end,
                        float *params_out, double *S_out)
{
    const or_line *L = o->L;
    const int P = o->P;
    const int32_t n_t = t_end - t_begin;
    int64_t total = 0;
#pragma omp parallel for collapse(2) schedule(dynamic, 4) reduction(+ : total)
    for (int32_t oi = 0; oi < n_out; ++oi) {
        for (int32_t tt = 0; tt < n_t; ++tt) {
            const int32_t j = cmp_out[oi], n0 = t_begin + tt;
            const uint64_t sample = (uint64_t)n0 + (uint64_t)L->nt * (uint64_t)j;
            const int np = or_pop_size(o->cfg, L->nt, n0);
            float lo[3], hi[3], pop[MAXNP * 3];
            double S[MAXNP];
            uint64_t w[4];
            or_sample_bounds(L, B, n0, lo, hi);
            for (int i = 0; i < np; ++i) {
                rng_words(seed, sample, 0, 0, (uint64_t)i, w);
                random_individual(w, P, lo, hi, pop + i * P);
                S[i] = objective(o, j, n0, pop + i * P, lo, hi);
            }
            int64_t ev = np + evolve(o, seed, sample, 0, j, n0, np, o->cfg->ng_f, lo, hi, pop, S);
            int b = best_index(S, np);
            const int64_t idx = (int64_t)oi * n_t + tt;
            for (int d = 0; d < P; ++d)
                params_out[idx * P + d] = pop[b * P + d];
            S_out[idx] = S[b];
            total += ev;
        }
    }
    return total;
}

static int64_t ens_sweep(const objective_ctx *o, const or_bounds *B, uint64_t seed,
                         const int32_t *cmp_out, int32_t n_out, int32_t t_begin, int32_t t_end,
                         float *params_out, double *S_out)
{
    const or_line *L = o->L;
    const or_de_cfg *cfg = o->cfg;
    const int P = o->P;
    const int32_t n_t = t_end - t_begin;
    const int64_t n_s = (int64_t)n_out * n_t;
    float *X = calloc((size_t)(n_s * P), sizeof(float)), *Y = calloc((size_t)(n_s * P), sizeof(float));
    double *XS = calloc((size_t)n_s, sizeof(double)), *YS = calloc((size_t)n_s, sizeof(double));
    const int n_stage = 1 + 2 * cfg->n_cycle;
    int64_t total = 0;

    const int32_t stride = cfg->n_skip + 1;
    for (int stage = 0; stage < n_stage; ++stage) {
        const int forward = (stage % 2) == 0;
        const int32_t init = stage == 0 ? 0 : (forward ? cfg->n_skip : (cfg->n_skip < 1 ? cfg->n_skip : 1));
        for (int32_t b0 = 0; b0 < n_out; b0 += cfg->n_bucket) {
            const int32_t nb = (n_out - b0) < cfg->n_bucket ? (n_out - b0) : cfg->n_bucket;
            for (int32_t k = 0; k < nb; ++k) {
                const int32_t pos = forward ? k : nb - 1 - k;
                const int32_t oi = b0 + pos;
                const int32_t prev = forward ? oi - 1 : oi + 1;
                const int32_t j = cmp_out[oi];
                int64_t step_total = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : step_total)
                for (int32_t tt = init; tt < n_t; tt += stride) {
                    const int32_t n0 = t_begin + tt;
                    const uint64_t sample = (uint64_t)n0 + (uint64_t)L->nt * (uint64_t)j;
                    const int np = stage == 0 ? or_pop_size(cfg, L->nt, n0) : cfg->np_bf;
                    const int ng = stage == 0 ? cfg->ng_f : cfg->ng_bf;
                    float lo[3], hi[3], pop[MAXNP * 3];
                    double S[MAXNP];
                    int scored[MAXNP];
                    uint64_t w[4];
                    or_sample_bounds(L, B, n0, lo, hi);
                    for (int i = 0; i < np; ++i) {
                        rng_words(seed, sample, (uint64_t)stage, 0, (uint64_t)i, w);
                        random_individual(w, P, lo, hi, pop + i * P);
                        scored[i] = 0;
                    }
                    const int64_t here = (int64_t)oi * n_t + tt;
                    if (stage == 0) {
                        if (cfg->inject && k > 0) {
                            const int64_t src = (int64_t)prev * n_t + tt;
                            memcpy(pop, Y + src * P, sizeof(float) * (size_t)P);
                            clamp_into(pop, P, lo, hi);
                        }
                    } else {
                        if (cfg->inject && tt > 0) {
                            memcpy(pop + 0 * P, X + (here - 1) * P, sizeof(float) * (size_t)P);
                            clamp_into(pop + 0 * P, P, lo, hi);
                        }
                        if (cfg->inject && tt < n_t - 1) {
                            memcpy(pop + 1 * P, X + (here + 1) * P, sizeof(float) * (size_t)P);
                            clamp_into(pop + 1 * P, P, lo, hi);
                        }
                        if (cfg->inject && k > 0) {
                            const int64_t src = (int64_t)prev * n_t + tt;
                            memcpy(pop + 2 * P, Y + src * P, sizeof(float) * (size_t)P);
                            clamp_into(pop + 2 * P, P, lo, hi);
                        }
                        /* the domain's own best so far, with its stored score */
                        memcpy(pop + 3 * P, X + here * P, sizeof(float) * (size_t)P);
                        S[3] = XS[here];
                        scored[3] = 1;
                    }
                    int64_t ev = 0;
                    for (int i = 0; i < np; ++i) {
                        if (!scored[i]) {
                            S[i] = objective(o, j, n0, pop + i * P, lo, hi);
                            ++ev;
                        }
                    }
                    ev += evolve(o, seed, sample, (uint64_t)stage, j, n0, np, ng, lo, hi, pop, S);
                    int bi = best_index(S, np);
                    memcpy(Y + here * P, pop + bi * P, sizeof(float) * (size_t)P);
                    YS[here] = S[bi];
                    step_total += ev;
                }
                if (stride > 1) {
                    /* interpolate the skipped samples of this trace */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : step_total)
                    for (int32_t tt = 0; tt < n_t; ++tt) {
                        if (tt >= init && (tt - init) % stride == 0)
                            continue;
                        const int32_t n0 = t_begin + tt;
                        const int64_t here = (int64_t)oi * n_t + tt;
                        const int32_t ta = tt > init ? tt - (tt - init) % stride : -1;
                        const int32_t tb_ = tt < init ? init : tt - (tt - init) % stride + stride;
                        const int32_t tb = tb_ < n_t ? tb_ : -1;
                        if (ta < 0 && tb < 0) {
                            /* nothing estimated in this stage: keep the stored individual */
                            memcpy(Y + here * P, X + here * P, sizeof(float) * (size_t)P);
                            YS[here] = XS[here];
                            continue;
                        }
                        float lo[3], hi[3], p[3];
                        or_sample_bounds(L, B, n0, lo, hi);
                        const float *pa = Y + ((int64_t)oi * n_t + (ta >= 0 ? ta : tb)) * P;
                        const float *pb = Y + ((int64_t)oi * n_t + (tb >= 0 ? tb : ta)) * P;
                        if (ta >= 0 && tb >= 0) {
                            const float wgt = (float)(tt - ta) / (float)(tb - ta);
                            for (int d = 0; d < P; ++d) {
                                const float diff = pb[d] - pa[d];
                                const float step = wgt * diff;
                                p[d] = pa[d] + step;
                            }
                        } else {
                            memcpy(p, pa, sizeof(float) * (size_t)P);
                        }
                        clamp_into(p, P, lo, hi);
                        const double Sp = objective(o, j, n0, p, lo, hi);
                        step_total += 1;
                        if (stage == 0 || Sp > XS[here]) {
                            memcpy(Y + here * P, p, sizeof(float) * (size_t)P);
                            YS[here] = Sp;
                        } else {
                            memcpy(Y + here * P, X + here * P, sizeof(float) * (size_t)P);
                            YS[here] = XS[here];
                        }
                    }
                }
                total += step_total;
            }
        }
        float *tp = X; X = Y; Y = tp;
        double *ts = XS; XS = YS; YS = ts;
    }
    memcpy(params_out, X, sizeof(float) * (size_t)(n_s * P));
    memcpy(S_out, XS, sizeof(double) * (size_t)n_s);
    free(X); free(Y); free(XS); free(YS);
    return total;
}

int64_t or_search(const or_line *L, const or_bounds *B, const or_de_cfg *cfg, uint64_t seed,
                  const int32_t *cmp_out, int32_t n_out, int32_t t_begin, int32_t t_end,
                  float *params_out, double *S_out)
{
    objective_ctx o = {L, cfg, L->op};
    if (!cfg->ens_enabled)
        return plain_de(&o, B, seed, cmp_out, n_out, t_begin, t_end, params_out, S_out);
    return ens_sweep(&o, B, seed, cmp_out, n_out, t_begin, t_end, params_out, S_out);
}
