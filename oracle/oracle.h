/*
 * FP64 CPU oracle for the coevolutionary traveltime-parameter search
 * (arXiv 2304.11399).  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the benchmark's CPU-baseline leg call it; the product library never
 * links, loads or calls anything here, and nothing here includes a header of
 * the product.
 *
 * Plain, slow, obviously-correct definitions in double precision.  Parameter
 * vectors of the evolutionary search are held in binary32 with every update
 * written out in binary32 operations (no fused multiply-add), because the
 * evolution's integer decisions (repair, crossover, argmax) must be taken in
 * the same precision as the device path; every semblance value is binary64.
 */
#ifndef ENS_ORACLE_H
#define ENS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A CMP-sorted prestack line plus the semblance configuration.
 * Section "Traveltime parameter search": f(p) = S(p; #data, #config) where
 * #data is the traces and geometry and #config the window, aperture and the
 * initial coordinate t0 (eq. Sf). */
typedef struct {
    const double *u;        /* [n_tr][nt] trace samples, sample n at time n*dt */
    int64_t n_tr;
    int32_t nt;
    double dt;
    const int64_t *cmp_ptr; /* [n_cmp+1] CSR row pointer, traces sorted by (CMP, offset) */
    int32_t n_cmp;
    double dx;              /* CMP spacing (m) */
    const double *offset;   /* [n_tr] full source-receiver offset h (m) */
    int32_t half_w;         /* window is 2*half_w+1 samples centred on the traveltime */
    int32_t op;             /* 1: CMP t^2 = t0^2 + C h^2 ; 3: CRS (A, B, C) */
    int32_t ap_lo, ap_hi;   /* midpoint half-aperture (CMPs) at t index 0 and nt-1 */
} or_line;

typedef struct {
    float lo[3], hi[3];
    uint32_t inv_t0_mask;   /* bit d: bound d is given for p_d*t0, divide by max(t0, dt) */
} or_bounds;

typedef struct {
    int32_t np_lo, np_hi;   /* NP_f at t index 0 and nt-1, linear in between */
    int32_t ng_f;           /* NG_f */
    int32_t np_bf, ng_bf;   /* NP_bf, NG_bf */
    int32_t n_cycle;        /* N_cycle */
    int32_t n_bucket;       /* traces per interactive domain */
    int32_t ens_enabled;    /* 0: every sample runs on its own (plain DE) */
    int32_t inject;         /* ENS sweep only: 0 disables every exchange of individuals */
    float F, CR;
    int32_t objective;      /* 0 semblance; 1 sphere mock; 2 needle mock */
    int32_t n_skip;         /* N_skip: time samples interpolated between estimated ones (0..2) */
    int32_t adapt;          /* 1: JADE control-parameter adaptation and archive (F, CR: initial means) */
} or_de_cfg;

/* OpenMP threads the oracle's parallel loops use, and setting them. */
int32_t or_num_threads(void);
void or_set_num_threads(int32_t n);

/* counter-based generator: Philox-4x64 with 10 rounds (Salmon et al., SC'11) */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

int32_t or_aperture(const or_line *L, int32_t n0);
int32_t or_pop_size(const or_de_cfg *cfg, int32_t nt, int32_t n0);
void or_sample_bounds(const or_line *L, const or_bounds *B, int32_t n0, float lo[3], float hi[3]);

/* Semblance of parameter vector p at ZO sample (CMP j, time index n0).
 * M_out: participating traces; margin_out: distance (samples) of the closest
 * aperture trace from a participation boundary. */
double or_semblance(const or_line *L, int32_t j, int32_t n0, const double *p,
                    int32_t *M_out, double *margin_out);
void or_semblance_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                        const double *params, double *S, int32_t *M, double *margin);
/* Sensitivity of S to the traveltimes: sum over the participating traces of
 * |dS/dtau_i| (tau in samples, M held fixed, right derivative at integer
 * traveltime).  A traveltime error of at most delta samples per trace moves S
 * by at most about delta times this sum (first order). */
void or_semblance_tau_l1_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                               const double *params, double *l1);
/* Distance of the participating traces' traveltimes from whole samples,
 * relative to the moveout: min_i |tau_i - round(tau_i)| / (1 + |tau_i - n0|)
 * (infinity when no trace takes part).  The interpolation has a kink at whole
 * samples, where the derivative in tau jumps; a computation whose traveltimes
 * carry a relative error may land on the other side of it. */
void or_kink_margin_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                          const double *params, double *out);
/* Gradient dS/dp (M held fixed, right derivative at integer traveltime). */
double or_semblance_grad(const or_line *L, int32_t j, int32_t n0, const double *p, double *g);
void or_semblance_grad_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                             const double *params, double *S, double *grad);

/* One generation's trial vectors from explicit generator words.
 * pop, trial: [np][P]; S: [np]; words: [np][4] (the four 64-bit outputs). */
void or_de_trial(int32_t np, int32_t P, const float *pop, const double *S, const uint64_t *words,
                 float F, float CR, const float *lo, const float *hi, float *trial);

/* JADE control parameters of one slot and one generation from the slot's
 * adaptation block w (Philox counter (sample, stage + 2^32, generation,
 * slot)): CR and F on the grid k / 2^24 (k_cr in [0, 2^24], k_f in
 * [1, 2^24]) and the archive position a replaced parent overwrites when the
 * archive is full. */
void or_jade_draws(const uint64_t w[4], double mu_cr, double mu_f, int32_t np, int32_t *k_cr,
                   int32_t *k_f, int32_t *a_idx);

/* The written-out binary64 series the JADE draws use: ln u (u > 0),
 * cos(2 pi t) for t in [0, 1) and tan(pi x) for x in (-1/2, 1/2). */
double or_jade_ln(double u);
double or_jade_cos_turns(double t);
double or_jade_tan_half_turn(double x);
/* y[i] = series which (0 ln, 1 cos_turns, 2 tan_half_turn) at x[i]. */
void or_jade_series_batch(int32_t which, int64_t n, const double *x, double *y);

/* ng JADE generations of one population of np members with explicit inputs,
 * through the same selection, archive and mean-update steps as the search:
 * pop [np][P], S [np] (in/out); de_words [ng][np][4] the slots' DE blocks;
 * the draws come from jade_words [ng][np][4] at the current means, or, when
 * jade_words is NULL, are given as draws [ng][np][3] = (k_cr, k_f, a_idx);
 * St [ng][np] the trial scores.  Initial means CR0, F0 and an empty archive.
 * Per generation: trials_out [ng][np][P], mu_out [ng][2] = (mu_CR, mu_F)
 * after its update, n_arch_out [ng] and archive_out [ng][np][P]. */
void or_jade_run(int32_t np, int32_t P, float *pop, double *S, int32_t ng, const uint64_t *de_words,
                 const uint64_t *jade_words, const int32_t *draws, const double *St, float F0, float CR0,
                 const float *lo, const float *hi, float *trials_out, double *mu_out, int32_t *n_arch_out,
                 float *archive_out);

/* One JADE generation's trial vectors: current-to-best/1 with the second
 * difference vector drawn from population plus archive (archive: [n_arch][P]),
 * per-slot F = k_f / 2^24 and CR = k_cr / 2^24; words: the slots' DE blocks. */
void or_jade_trial(int32_t np, int32_t P, const float *pop, const double *S, const float *archive,
                   int32_t n_arch, const uint64_t *words, const int32_t *k_f, const int32_t *k_cr,
                   const float *lo, const float *hi, float *trial);

/* Whole search.  cmp_out: [n_out] output CMPs; time indices [t_begin, t_end).
 * params_out: [n_out][n_t][P]; S_out: [n_out][n_t].  Returns evaluations. */
int64_t or_search(const or_line *L, const or_bounds *B, const or_de_cfg *cfg, uint64_t seed,
                  const int32_t *cmp_out, int32_t n_out, int32_t t_begin, int32_t t_end,
                  float *params_out, double *S_out);

/* Gradient-ascent polish (Adam on box-normalised coordinates), best-so-far kept. */
void or_polish(const or_line *L, const or_bounds *B, int64_t n, const int32_t *cmp,
               const int32_t *t, const float *p_in, double lr, int32_t steps,
               double *p_out, double *S_out);

/* Per-trace scaled reduced-precision storage: scale = the smallest power of
 * two at or above max|u| (1 if the trace is all zero), q =
 * round-to-nearest-even(u / scale) (the quotient is exact in binary32). */
void or_quantize(const float *u, int64_t n_tr, int32_t nt, int32_t dtype /*1 f16, 2 bf16*/,
                 uint16_t *q, float *scale);
double or_half_to_double(uint16_t h);
double or_bf16_to_double(uint16_t h);

/* Zero-offset stack: mean over the participating traces of the interpolated
 * amplitude at each trace's traveltime (0 when none takes part). */
double or_stack(const or_line *L, int32_t j, int32_t n0, const double *p, int32_t *M_out);
void or_stack_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                    const double *params, double *out, int32_t *M);
/* Root mean square of a panel. */
double or_rms(const double *x, int64_t n);

/* Reference maximum of S per sample: uniform grid then local refinement. */
void or_sref(const or_line *L, const or_bounds *B, int64_t n, const int32_t *cmp,
             const int32_t *t, const int32_t *grid /*[3] points per axis*/, int32_t n_refine,
             double *S_ref, double *p_ref);

#ifdef __cplusplus
}
#endif
#endif
