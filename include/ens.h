/*
 * libens — windowed-semblance traveltime-parameter search with evolution by
 * neighbourhood similarity (ENS), for AMD Instinct MI355X (gfx950).
 *
 * Method: arXiv 2304.11399.  For every zero-offset output sample (t, tr) the
 * library searches the traveltime-operator parameters that maximise the
 * semblance of the data along the operator (section "Traveltime parameter
 * search", eqs. f, S, Sf); each sample runs a differential evolution
 * (section "JADE applied to traveltime parameter search") and, with ENS
 * enabled, best individuals are exchanged between neighbouring samples in a
 * forward exploration sweep followed by backward/forward exploitation sweeps
 * over the traces of each interactive domain (sections "Information
 * propagation" and "Evolution by neighborhood similarity").
 *
 * Operators (h = full source-receiver offset, dm = midpoint displacement of
 * a trace's CMP from the output CMP, t0 = n0 dt):
 *     ENS_OP_CMP (1 parameter C):          t^2 = t0^2 + C h^2
 *     ENS_OP_CRS (3 parameters A, B, C):   t^2 = (t0 + A dm)^2 + B t0 dm^2 + C t0 h^2
 *
 * Semblance of M participating traces (t^2 >= 0 and 0 <= t/dt <= nt-1) over
 * the window k = -w..w around each trace's traveltime tau = t/dt = n + f:
 *     a_ik = (1-f) u_i[n+k] + f u_i[n+k+1]   (samples outside the trace read 0)
 *     S = sum_k (sum_i a_ik)^2 / (M sum_k sum_i a_ik^2),  S = 0 if M = 0 or the
 *     energy is 0.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE pointers unless marked "host".  The caller owns
 *    every buffer it passes; the library never frees them and keeps no
 *    pointer to them after the call returns, except that ens_bind copies the
 *    traces into its own store.
 *  - Work is ordered on the context's stream.  Device outputs are valid once
 *    that stream has been synchronised; host outputs (counters) are written
 *    before the call returns (those calls synchronise the stream once).
 *  - Arguments are validated on the host before anything is launched; on an
 *    error nothing is written to any output, the call returns a negative
 *    ens_status and ens_last_error(ctx) describes the problem.  No C++
 *    exception crosses this interface.  A context is used by one host thread
 *    at a time.
 *  - Every struct begins with struct_size = sizeof(struct); a smaller value
 *    is rejected with ENS_E_INVALID.
 */
#ifndef ENS_H
#define ENS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ENS_OK = 0,
    ENS_E_INVALID = -1,     /* null pointer, bad dtype/op, inconsistent sizes, struct_size */
    ENS_E_RANGE = -2,       /* even or too large window, NP < 4 or > 64, NP_bf < 5, lo >= hi,
                               n_skip outside 0..2 or without ENS, index out of range */
    ENS_E_HIP = -3,         /* a HIP runtime call failed (message has the HIP error string) */
    ENS_E_OOM = -4,         /* device allocation failed */
    ENS_E_UNSUPPORTED = -5, /* valid request the library does not implement */
    ENS_E_STATE = -6        /* call needs ens_bind first */
} ens_status;

enum { ENS_DTYPE_F32 = 0, ENS_DTYPE_F16 = 1, ENS_DTYPE_BF16 = 2 };
enum { ENS_OP_CMP = 1, ENS_OP_CRS = 3 };
enum { ENS_MAX_HALF_WINDOW = 7 };       /* window W = 2w+1 <= 15 */
enum { ENS_MAX_POP = 64 };

typedef struct ens_ctx ens_ctx;

/* Trace samples, read once by ens_bind (#data of eq. Sf).  data: device
 * [n_traces][ld], sample n of trace i at data[i*ld + n], time n*dt, of type
 * data_dtype:
 *  - ENS_DTYPE_F32: binary32 samples.  store_dtype chooses the library's
 *    own storage: F32 keeps binary32; F16/BF16 keep q_i[n] =
 *    round-to-nearest-even(u_i[n] / s_i) with the per-trace scale s_i the
 *    smallest power of two at or above max_n |u_i[n]| (1 for an all-zero
 *    trace; the quotient is exact), plus the binary32 samples for the
 *    binary64 re-scoring and the stack.
 *  - ENS_DTYPE_F16 / ENS_DTYPE_BF16: caller-quantised 16-bit samples
 *    (binary16 / bfloat16 bit patterns) with scale (device [n_traces]) the
 *    per-trace scales, each a positive power of two (ens_quantize writes
 *    such scales; others are rejected with ENS_E_RANGE): the samples are
 *    s_i q_i[n].  store_dtype must be data_dtype (searched in 16 bits) or F32
 *    (the exact dequantised samples are stored).  master (optional, device
 *    [n_traces][ld] binary32): the samples the binary64 re-scoring and the
 *    stack read; NULL: the dequantised samples.
 * scale and master are ignored for binary32 data.  Samples must be finite.
 * nt is at most 2^20; searched in binary16 (store_dtype F16) at most
 * ENS_MAX_NT_F16: the binary16 windows round each traveltime to the grid
 * 2^(lb-23) samples, 2^lb the smallest power of two >= max(4096, nt + 16)
 * (2^-11 samples up to 4080 samples, 2^-10 up to 8176, 2^-9 up to 16368);
 * longer records are refused (ENS_E_UNSUPPORTED): store them as binary32 or
 * bfloat16, whose windows take exact traveltimes. */
enum { ENS_MAX_NT_F16 = 16368 };
typedef struct {
    uint32_t struct_size;
    const void *data;
    int64_t n_traces;
    int32_t nt;
    int64_t ld;
    float dt;
    int32_t store_dtype;
    int32_t data_dtype;
    const float *scale;
    const float *master;
} ens_traces;

/* Acquisition geometry, host arrays.  Traces sorted by (CMP, offset);
 * cmp_ptr[c] .. cmp_ptr[c+1]-1 are the traces of CMP c, cmp_ptr[0] = 0,
 * cmp_ptr[n_cmp] = n_traces, non-decreasing.  offset: full offset (m) per
 * trace.  dx: CMP spacing (m); dm = (c - j) dx. */
typedef struct {
    uint32_t struct_size;
    const int64_t *cmp_ptr;  /* host [n_cmp+1] */
    int32_t n_cmp;
    float dx;
    const float *offset;     /* host [n_traces] */
} ens_geometry;

/* Semblance configuration (#config of eq. Sf): operator, window length and
 * midpoint half-aperture in CMPs, ap_lo at time index 0 and ap_hi at nt-1,
 * a(n0) = floor(ap_lo + (ap_hi - ap_lo) n0 / (nt-1) + 1/2). */
typedef struct {
    uint32_t struct_size;
    int32_t op;
    int32_t window;          /* odd, <= 2*ENS_MAX_HALF_WINDOW+1 */
    int32_t ap_lo, ap_hi;
} ens_sem_cfg;

/* Output grid: output CMPs (host list; NULL = all CMPs in order) and time
 * indices [t_begin, t_end).  ZO sample id = t + nt*cmp.  Results are laid out
 * [n_cmp_out][t_end - t_begin] with t fastest. */
typedef struct {
    uint32_t struct_size;
    const int32_t *cmp_out;  /* host [n_cmp_out] or NULL */
    int32_t n_cmp_out;
    int32_t t_begin, t_end;
} ens_t0_grid;

/* Parameter box.  Bit d of inv_t0_mask set: bounds d are given for p_d t0 and
 * are divided per sample by max(t0, dt) (binary32: lo_d / max(n0*dt, dt)). */
typedef struct {
    uint32_t struct_size;
    float lo[3], hi[3];
    uint32_t inv_t0_mask;
} ens_bounds;

/* Search configuration.  NP_f(n0) = floor(np_lo + (np_hi-np_lo) n0/(nt-1) + 1/2).
 * ens_enabled = 0: every sample evolves on its own (NP_f, NG_f) — the
 * per-domain search the paper compares against.  ens_enabled = 1: ENS with
 * buckets of n_bucket consecutive output CMPs, stage 0 (NP_f, NG_f) and
 * n_cycle backward/forward cycles (NP_bf, NG_bf); inject = 0 disables every
 * exchange between samples.  n_skip (0, 1 or 2; ENS only): each stage
 * searches every (n_skip+1)-th time sample, from offset 0 in the first
 * forward sweep, min(1, n_skip) in backward sweeps and n_skip in later forward
 * sweeps; the other samples take the clamped linear interpolation in t of
 * that stage's estimates (the nearest one past either end), scored once, and
 * in stages after the first keep their stored individual when it scores
 * higher (sections "The performance-quality trade-off by an interpolation
 * process" and "Evolution by neighborhood similarity", eq. for
 * the ENS evaluation count).  F, CR: fixed mutation factor
 * and crossover rate.  adapt = 1: JADE with archive in every domain (the
 * paper's per-domain engine, sections "Selection" and "Evolution by
 * neighborhood similarity"; its rules are JADE's published ones): per slot
 * and generation CR ~ N(mu_CR, 0.1) clipped to [0, 1] and F ~ Cauchy(mu_F,
 * 0.1), cut to 1, redrawn where not positive, both on the grid k / 2^24;
 * the second difference vector's minuend drawn from population plus
 * archive of replaced parents (at most NP); after each generation the means
 * move 10% toward the arithmetic mean of the successful CR and the Lehmer
 * mean of the successful F; F and CR give the initial means (F in (0, 1]).  polish_steps > 0: that many Adam steps of learning
 * rate polish_lr on box-normalised coordinates per winner, keeping the best
 * point.  rescore_fp64: also write the binary64 semblance of each winner,
 * computed from the binary32 copy of the traces. */
typedef struct {
    uint32_t struct_size;
    int32_t np_lo, np_hi;
    int32_t ng_f;
    int32_t np_bf, ng_bf;
    int32_t n_cycle;
    int32_t n_skip;
    int32_t n_bucket;
    int32_t ens_enabled;
    int32_t inject;
    float F, CR;
    int32_t polish_steps;
    float polish_lr;
    int32_t rescore_fp64;
    int32_t adapt;
} ens_de_cfg;

/* Search outputs (device, [n_cmp_out][n_t][P] and [n_cmp_out][n_t]); S64 and
 * S_pre_polish may be NULL.  n_evals, sum_m (host) receive the evaluation
 * count and the total of participating traces over all evaluations. */
typedef struct {
    uint32_t struct_size;
    float *params;
    float *S;
    double *S64;
    float *S_pre_polish;
    int64_t n_evals;
    int64_t sum_m;
} ens_result;

/* A batch of candidates: output CMP, time index and parameters [n][P]
 * (device).  Throughput is best when consecutive candidates share a CMP. */
typedef struct {
    uint32_t struct_size;
    int64_t n;
    const int32_t *cmp;
    const int32_t *t;
    const float *params;
} ens_candidates;

/* Search-kernel launch shape.  Zero fields are chosen by measurement: the
 * first search of a given shape times its first launch of each kernel kind,
 * first for every slice count (1, 2, 4, 8) at the first free item order and
 * register budget, then for the other orders and budgets at the fastest count,
 * then (exploration, where offered) packed workgroups of 2, 4 and 8 waves at
 * the best order and budget so far and the other orders and budgets at the
 * fastest width (a launch under 5 ms timed three times, the fastest counting),
 * and keeps the fastest for later searches of that shape (the generation
 * count does not enter the shape).  Measured shapes persist in a text file:
 * ENS_TUNE_CACHE if set ("off": none), else ens_tune_cache.txt beside the
 * library, keyed by device (architecture and compute units) and shape. */
typedef struct {
    uint32_t struct_size;
    int32_t waves_per_sample_group;  /* trace slices per population (1, 2, 4, 8); 0: measure */
    int32_t use_graph;               /* 1: replay the trace-step launches as a HIP graph */
    int32_t collect_timing;          /* 1: time every search launch with HIP events */
    int32_t item_order;              /* 0: measure; 1: XCD-contiguous (bucket, t) order;
                                        2: costliest items first, dealt round-robin;
                                        3: XCD-contiguous shares, costliest first in each */
    int32_t occupancy;               /* 0: measure; 1: registers as compiled (4 waves per SIMD);
                                        2: held to 64 registers (8 waves per SIMD) */
    int32_t packing;                 /* exploration launches with fixed F and CR (plain search,
                                        ENS stage 0): 2, 4 or 8 lays the populations of
                                        consecutive samples end to end over that many waves
                                        (one evaluation per lane, no trace slices;
                                        waves_per_sample_group then applies to the
                                        exploitation launches only); 1: one population per
                                        lane group; 0: measured with the other fields where
                                        under 90% of the lanes would carry a member (when
                                        waves_per_sample_group and item_order are 0 too),
                                        else 1.  A packed launch gives the results of one
                                        population per lane group with one slice, bit for
                                        bit; slice counts above 1 change the order of the
                                        window sums. */
    int32_t gather;                  /* 0: windows read directly from the rows; 1: binary32
                                        rows staged per trace in LDS (the column range every
                                        window may read, bounded from the samples' boxes) and
                                        the windows read from LDS, for searches with fixed F
                                        and CR outside packed workgroups.  Same results bit
                                        for bit; measured slower on the CRS lines. */
} ens_tuning;

/* Work and device time of the last ens_search, per kernel kind:
 * [0] exploration launches (plain evolution, or ENS stage 0),
 * [1] exploitation launches (ENS backward/forward stages),
 * [2] gradient polish, [3] binary64 re-scoring.
 * evals / sum_m: semblance evaluations and participating traces summed over
 * them (for [2]: forward evaluations of the polish).  device_ms is the sum of
 * the launches' event-timed durations when collect_timing was set, else 0. */
typedef struct {
    uint32_t struct_size;
    int64_t launches[4];
    int64_t evals[4];
    int64_t sum_m[4];
    double device_ms[4];
    int32_t waves_used[2];   /* trace slices chosen for kinds [0] and [1] */
    int32_t order_used[2];   /* item order chosen (1 or 2) for kinds [0] and [1] */
    int32_t dense_used[2];   /* 1 if the 64-register variant was chosen */
    double tune_ms;          /* device time spent measuring launch shapes in this call */
    int32_t packed_used;     /* waves of a packed exploration workgroup, 0 if not packed */
} ens_stats;

/* ---- context ----------------------------------------------------------- */

/* Create a context on the current HIP device ordering its work on `stream`
 * (a hipStream_t; NULL = the null stream). */
ens_status ens_ctx_create(ens_ctx **out, void *stream);
void ens_ctx_destroy(ens_ctx *ctx);
/* Message of the last failing call on ctx (empty string if none). */
const char *ens_last_error(const ens_ctx *ctx);
/* Library version string. */
const char *ens_version(void);
ens_status ens_set_tuning(ens_ctx *ctx, const ens_tuning *tuning);
/* Statistics of the last successful ens_search on ctx (host struct). */
ens_status ens_last_stats(const ens_ctx *ctx, ens_stats *out);

/* ---- data --------------------------------------------------------------- */

/* Bind #data and #config (eq. Sf): copies the traces into the library's
 * padded store (quantising them if asked) and uploads the geometry. */
ens_status ens_bind(ens_ctx *ctx, const ens_traces *traces, const ens_geometry *geometry,
                    const ens_sem_cfg *sem);

/* Per-trace scaled quantisation of [n_traces][ld] binary32 samples into
 * q: device [n_traces][nt] uint16 (binary16 or bfloat16 bits) and scale:
 * device [n_traces], the smallest power of two at or above each trace's
 * largest magnitude (the rule ens_bind applies; its output is valid 16-bit
 * input for ens_bind). */
ens_status ens_quantize(ens_ctx *ctx, const float *data, int64_t n_traces, int32_t nt, int64_t ld,
                        int32_t dtype, uint16_t *q, float *scale);

/* ---- the search --------------------------------------------------------- */

/* Search every sample of t0_grid over the bound data (section "Traveltime
 * parameter search": maximise f(p) = S(p; #data, #config) within the box per
 * sample). */
ens_status ens_search_bound(ens_ctx *ctx, const ens_t0_grid *t0_grid, const ens_bounds *bounds,
                            const ens_de_cfg *de_cfg, uint64_t seed, ens_result *out);

/* The whole search in one call: ens_bind(traces, geometry, sem) followed by
 * ens_search_bound(t0_grid, bounds, de_cfg, seed) — f(p) = S(p; #data,
 * #config) maximised per sample, with #data = (traces, geometry) and #config =
 * (sem, t0_grid) (eq. Sf).  Results and errors as for those two calls; the
 * data stay bound to ctx afterwards. */
ens_status ens_search(ens_ctx *ctx, const ens_traces *traces, const ens_geometry *geometry,
                      const ens_sem_cfg *sem, const ens_t0_grid *t0_grid, const ens_bounds *bounds,
                      const ens_de_cfg *de_cfg, uint64_t seed, ens_result *out);

/* ---- the objective and its adjoint --------------------------------------- */

/* f(p) for a batch: S_out[n] (device); M_out[n] (device, may be NULL)
 * receives the participating-trace counts.  Uses the bound store. */
ens_status semblance_eval(ens_ctx *ctx, const ens_candidates *cands, float *S_out, int32_t *M_out);

/* Binary64 semblance from the binary32 copy of the traces: S_out[n] (device). */
ens_status semblance_eval64(ens_ctx *ctx, const ens_candidates *cands, double *S_out);

/* dparams_out[n][P] = dS[n] * dS/dp through the interpolated gather, with M
 * held fixed and the right derivative at integer traveltimes (device). */
ens_status semblance_backward(ens_ctx *ctx, const ens_candidates *cands, const float *dS,
                              float *dparams_out);

/* ---- outputs for inspection --------------------------------------------- */

/* Zero-offset stack of every sample of t0_grid along the operator given by
 * params (device [n_out][n_t][P], as ens_search writes them): the mean over
 * the traces that take part in that sample's semblance of the amplitude
 * interpolated at each trace's traveltime, 0 for an empty fold, computed from
 * the binary32 copy of the traces (sections "Traveltime parameter search",
 * "Qualitative analysis").  stack_out: device [n_out][n_t].  If S (device
 * [n_out][n_t], e.g. ens_result.S) and coherence_rms (host) are both given,
 * *coherence_rms receives sqrt(sum S^2 / (n_out n_t)) in binary64, the RMS of
 * the coherence panel (section "Quantitative analysis"); the call then waits
 * for the stream.  Errors as for ens_search's grid. */
ens_status ens_stack(ens_ctx *ctx, const ens_t0_grid *t0_grid, const float *params, float *stack_out,
                     const float *S, double *coherence_rms);

/* ens_stack for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same outputs from the same
 * kernels, with the output-CMP list and the
 * coherence RMS kept in a static per-device scratch array of 256 B + 4 B x
 * ENS_NOALLOC_MAX_CMPS (held by each GPU the library runs on until the
 * process ends) instead of context workspace.  No hipMalloc, hipFree or
 * allocating routine is called.  At most ENS_NOALLOC_MAX_CMPS output CMPs
 * (more: ENS_E_RANGE, nothing launched).  Every call on one GPU uses that
 * GPU's one array, so calls that overlap on a GPU (from other contexts,
 * threads or streams) race; calls ordered on one stream do not.  Waits for
 * the stream before returning (the RMS is returned on the host), so it is
 * not meant to be recorded into a stream capture.  Arguments and errors
 * otherwise as ens_stack. */
enum { ENS_NOALLOC_MAX_CMPS = 65536 };
ens_status ens_stack_noalloc(ens_ctx *ctx, const ens_t0_grid *t0_grid, const float *params, float *stack_out,
                             const float *S, double *coherence_rms);

/* ---- checks of the device building blocks -------------------------------- */

/* Philox-4x64-10 blocks (Salmon et al., SC'11) for n counters (device
 * [n][4] uint64) under key (device [2]): out device [n][4]. */
ens_status ens_philox(ens_ctx *ctx, int64_t n, const uint64_t *counters, const uint64_t *key,
                      uint64_t *out);

/* JADE's per-slot draws for n adaptation blocks (device words [n][4], the
 * Philox outputs for counter (sample, stage + 2^32, generation, slot)) at
 * means mu_cr, mu_f: k_cr, k_f, a_idx device [n] (CR = k_cr / 2^24,
 * F = k_f / 2^24, the archive position for a full archive of np entries).
 * The search kernels use the same device routine. */
ens_status ens_jade_draws(ens_ctx *ctx, int64_t n, const uint64_t *words, double mu_cr, double mu_f,
                          int32_t np, int32_t *k_cr, int32_t *k_f, int32_t *a_idx);

/* One generation's trial vectors of the evolution for n_pop independent
 * populations of size np (device pop [n_pop*np][P], S [n_pop*np], words
 * [n_pop*np][4] generator outputs, lo/hi [n_pop][P]): trial out
 * [n_pop*np][P].  The search kernels use the same device routine. */
ens_status ens_de_trial(ens_ctx *ctx, int32_t n_pop, int32_t np, int32_t P, const float *pop,
                        const float *S, const uint64_t *words, float F, float CR,
                        const float *lo, const float *hi, float *trial);

#ifdef __cplusplus
}
#endif
#endif
