// Argument blocks and launch wrappers shared by kernels.hip and api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ens {

struct TraceMeta;

// Bound trace store and per-time tables.
struct StoreView {
    const void *store;        // [n_tr][ld] padded rows, sample 0 at column PAD
    int64_t ld;               // row stride in elements
    int32_t copy1;            // 16-bit rows: element offset of the copy shifted by one sample (else 0)
    const float *scale;       // [n_tr] per-trace scale, or nullptr for binary32 storage
    const TraceMeta *meta;    // [n_tr]
    const int64_t *cmp_ptr;   // [n_cmp+1]
    int32_t n_cmp;
    int32_t nt;
    float dt, dx;
    const int32_t *ap_tab;    // [nt] half-aperture per time index
    // binary16 windows (see accum_trace_f16)
    const uint32_t *wsc16;    // [n_tr] per-trace weight scale 2^(e_i - g) as a pair of binary16
    float h16_kq;             // B + PAD - W/2: tau + h16_kq lies in [B, 2B), spacing = weight grid
    uint32_t h16_bbits;       // bit pattern of the binary32 B
    uint32_t h16_shift;       // (bits(floor(tau + h16_kq)) - h16_bbits) >> h16_shift = 2 * column
    float tau_max;            // nt - 1
};

struct CandView {
    int64_t n;
    const int32_t *cmp;
    const int32_t *t;
    const float *params;      // [n][P]
};

// One launch of the evolution: either every sample of the grid evolving on
// its own (plain), or the trace steps [k_begin, k_end) of one ENS stage in
// every bucket.
struct SearchArgs {
    StoreView sv;
    const int32_t *cmp_out;   // [n_out] output CMPs
    int32_t n_out, t_begin, n_t;
    const float *lo_tab, *hi_tab;  // [nt][3] per-time boxes
    const int4 *items;        // work items {output index or bucket, first t,
                              //  samples | stride << 8, NP}
    int32_t n_items;
    int32_t plain, stage, k_begin, k_end, forward, n_bucket, ng, inject, nsl;
    int32_t xcd_order;        // 1: deal consecutive items to one XCD; 0: items in block order
    uint64_t seed;
    float F, CR;              // fixed F and CR, or JADE's initial means
    uint64_t cr_thr;          // crossover draw threshold ceil(CR 2^32)
    int32_t adapt;            // 1: JADE control-parameter adaptation and archive
    const float *Xp, *XS;     // previous stage state [n_out][n_t][P], [n_out][n_t]
    float *Yp, *YS;           // this stage's state
    unsigned long long *counters;  // [2 KIND] evaluations, [2 KIND + 1] participating traces
    unsigned long long *progress;  // sweep steps finished in this launch (zeroed before it), or null
    // packed exploration (k_search_packed): populations laid end to end over
    // the nsl waves of a workgroup; items {group, first t, samples | stride << 8, 0}
    int32_t packed;
    const int32_t *np_tab;    // [nt] NP_f per time index
    // LDS-staged windows (binary32 rows): per trace step a table of each
    // aperture trace's column range over the workgroup's boxes, then per trace
    // the range staged by coalesced loads and the windows read from LDS
    int32_t tiles;
    int32_t tile_cap;         // table entries: the most traces any aperture union holds
};

// binary32 samples one staged trace may span (longer ranges read directly)
constexpr int TILE_STAGE_MAX = 192;

// samples one packed workgroup may hold (populations have at least 4 members)
constexpr int PACK_MAX_SAMPLES_PER_WAVE = 16;

// Interpolation of the samples a stage skipped (time-sample skipping).
struct InterpArgs {
    StoreView sv;
    const int32_t *cmp_out;
    int32_t n_out, t_begin, n_t;
    const float *lo_tab, *hi_tab;
    int32_t stride, init, stage, kind;
    const float *Xp, *XS;     // previous stage state (stage > 0)
    float *Yp, *YS;           // this stage's state, in/out
    unsigned long long *counters;
};

struct PolishArgs {
    StoreView sv;
    const int32_t *cmp_out;
    int32_t n_out, t_begin, n_t;
    const float *lo_tab, *hi_tab;
    float *params;            // [n_out][n_t][P] in/out
    float *S;                 // [n_out][n_t] in/out
    float *S_pre;             // optional copy of the incoming S
    int32_t steps;
    float lr;
    unsigned long long *counters;  // [4] forward evaluations, [5] participating traces
};

// launch wrappers (return hipSuccess or the launch error)
hipError_t launch_store_f32(const float *src, int64_t ld_in, int64_t n_tr, int32_t nt, int64_t ld,
                            float *dst, hipStream_t s);
// dual: each output row is two rows of ld_out, the second shifted by one sample;
// exp_out (optional): per-trace scale exponent (INT32_MIN for a zero trace)
hipError_t launch_quantize(const float *src, int64_t ld_in, int64_t n_tr, int32_t nt, int32_t dtype,
                           uint16_t *dst, int64_t ld_out, int32_t col0, float *scale, bool dual,
                           int32_t *exp_out, hipStream_t s);
// caller-quantised 16-bit rows into the dual padded layout (+ optional dequantised binary32 master)
hipError_t launch_store16(const uint16_t *src, int64_t ld_in, int64_t n_tr, int32_t nt, int32_t dtype,
                          const float *scale, uint16_t *dst, int64_t ld_out, float *master, int32_t *exp_out,
                          hipStream_t s);
// relative weight scales of a 16-bit store from the exponents k_quantize wrote
hipError_t launch_relscale(const int32_t *e, int64_t n_tr, float *rel, uint32_t *wsc16, hipStream_t s);
hipError_t launch_eval(int op, int dtype, int window, const StoreView &sv, const CandView &cv,
                       float *S, int32_t *M, hipStream_t s);
hipError_t launch_eval64(int op, int window, const StoreView &sv_f32, const CandView &cv, double *S,
                         hipStream_t s);
hipError_t launch_eval64_grid(int op, int window, const StoreView &sv_f32, const int32_t *cmp_out,
                              int32_t n_out, int32_t t_begin, int32_t n_t, const float *params,
                              double *S, hipStream_t s);
hipError_t launch_backward(int op, int dtype, int window, const StoreView &sv, const CandView &cv,
                           const float *dS, float *g, hipStream_t s);
hipError_t launch_stack(int op, const StoreView &sv_f32, const int32_t *cmp_out, int32_t n_out, int32_t t_begin,
                        int32_t n_t, const float *params, float *out, hipStream_t s);
hipError_t launch_rms(const float *x, int64_t n, double *out, hipStream_t s);
hipError_t launch_search(int op, int dtype, int window, int kind, int dense, const SearchArgs &a,
                         int32_t n_blocks, hipStream_t s);
hipError_t launch_polish(int op, int dtype, int window, const PolishArgs &a, hipStream_t s);
hipError_t launch_interp(int op, int dtype, int window, const InterpArgs &a, hipStream_t s);
hipError_t launch_philox(int64_t n, const uint64_t *ctr, const uint64_t *key, uint64_t *out,
                         hipStream_t s);
hipError_t launch_jade_draws(int64_t n, const uint64_t *words, double mu_cr, double mu_f, int32_t np,
                             int32_t *k_cr, int32_t *k_f, int32_t *a_idx, hipStream_t s);
hipError_t launch_de_trial(int32_t n_pop, int32_t np, int32_t P, const float *pop, const float *S,
                           const uint64_t *words, float F, uint64_t cr_thr, const float *lo,
                           const float *hi, float *trial, hipStream_t s);

bool window_supported(int window);

}  // namespace ens
