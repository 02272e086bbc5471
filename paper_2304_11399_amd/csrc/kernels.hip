// HIP kernels of libens (gfx950) and their launch wrappers.
#include "device.h"
#include "launch.h"

namespace ens {

// ---------------------------------------------------------------------------
// trace store

// Copy [n_tr][ld_in] binary32 samples into the padded store [n_tr][ld]
// (PAD zeros, nt samples, zeros to the row end).  One workgroup per trace.
__global__ void k_store_f32(const float *__restrict__ src, int64_t ld_in, int32_t nt, int64_t ld,
                            float *__restrict__ dst)
{
    const int64_t i = blockIdx.x;
    for (int64_t n = threadIdx.x; n < ld; n += blockDim.x) {
        const int64_t m = n - PAD;
        dst[i * ld + n] = (m >= 0 && m < nt) ? src[i * ld_in + m] : 0.0f;
    }
}

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((b >> 16) | 0x40u);
    return static_cast<uint16_t>((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_bits(float x)
{
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
}

// One workgroup (256 threads) per trace: scale = max|u| (1 when the trace is
// zero), q = RNE(u / scale).  Output row stride ld_out with the first sample
// at column col0; when col0 > 0 the whole padded row is written.
// dual: the row is written twice, [0, ld_out) as laid out and
// [ld_out, 2 ld_out) shifted left by one sample (column c holds column c + 1).
__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ src, int64_t ld_in,
                                                  int32_t nt, int32_t dtype,
                                                  uint16_t *__restrict__ dst, int64_t ld_out,
                                                  int32_t col0, float *__restrict__ scale_out, int32_t dual)
{
    __shared__ float part[256 / WAVE];
    const int64_t i = blockIdx.x;
    const float *row = src + i * ld_in;
    float m = 0.0f;
    for (int32_t n = threadIdx.x; n < nt; n += blockDim.x) m = fmaxf(m, fabsf(row[n]));
    for (int off = WAVE / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = m;
    __syncthreads();
    float s = 0.0f;
    for (int w = 0; w < static_cast<int>(blockDim.x / WAVE); ++w) s = fmaxf(s, part[w]);
    if (s == 0.0f) s = 1.0f;
    if (threadIdx.x == 0) scale_out[i] = s;
    uint16_t *out = dst + i * (dual ? 2 * ld_out : ld_out);
    const int64_t row_len = dual ? 2 * ld_out : (col0 > 0 ? ld_out : nt);
    for (int64_t n = threadIdx.x; n < row_len; n += blockDim.x) {
        const int64_t c = n < ld_out ? n : n - ld_out + 1;
        const int64_t m2 = c - col0;
        uint16_t q = 0;
        if (m2 >= 0 && m2 < nt) {
            const float x = row[m2] / s;
            q = dtype == DT_F16 ? f32_to_f16_bits(x) : f32_to_bf16_bits(x);
        }
        out[n] = q;
    }
}

// ---------------------------------------------------------------------------
// wave helpers

template <typename T>
__device__ __forceinline__ T wave_min(T v)
{
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off, WAVE);
        v = o < v ? o : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off, WAVE);
        v = o > v ? o : v;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Union of the lanes' aperture CMP ranges (wave-uniform; empty: c_hi < c_lo).
__device__ __forceinline__ void wave_cmp_range(const StoreView &sv, int32_t j, int32_t ap, bool live,
                                               int32_t &c_lo, int32_t &c_hi)
{
    int32_t lo = j - ap < 0 ? 0 : j - ap;
    int32_t hi = j + ap > sv.n_cmp - 1 ? sv.n_cmp - 1 : j + ap;
    if (!live) {
        lo = 0x7fffffff;
        hi = -1;
    }
    c_lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    c_hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
}

template <typename R>
__device__ __forceinline__ R h2_of(const ENS_CONST_AS TraceMeta *meta, int32_t i)
{
    if constexpr (sizeof(R) == 8) {
        const R h = static_cast<R>(meta[i].h);
        return h * h;
    } else {
        return meta[i].h2;
    }
}

// Window sums of one candidate over the traces of CMPs c_lo..c_hi; in each
// CMP the traces first, first + step, first + 2 step, ... (two per step of
// the loop, so that their gathers are in flight together).
template <int DT, int W, bool SCALED, typename R>
__device__ __forceinline__ void accumulate_cmps(const StoreView &sv, const Cand<R> &cand, int32_t c_lo,
                                                int32_t c_hi, int32_t first, int32_t step,
                                                Acc<W, R> &acc)
{
    using T = typename Store<DT>::T;
    const T *store = static_cast<const T *>(sv.store);
    const ENS_CONST_AS int64_t *cmp_ptr = const_view(sv.cmp_ptr);
    const ENS_CONST_AS TraceMeta *meta = const_view(sv.meta);
    const ENS_CONST_AS float *scale = const_view(sv.scale);
    const R dx = static_cast<R>(sv.dx);
    const uint32_t row_bytes = static_cast<uint32_t>(sv.ld * static_cast<int64_t>(sizeof(T)));
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const CmpTerm<R> ct = cmp_term(cand, c, dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
        int32_t i = static_cast<int32_t>(cmp_ptr[c]) + first;
        for (; i + step < i1; i += 2 * step) {
            const int32_t i2 = i + step;
            accum_trace<DT, W, SCALED>(acc, cand, ct, h2_of<R>(meta, i),
                                       store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes,
                                       SCALED ? scale[i] : 1.0f);
            accum_trace<DT, W, SCALED>(acc, cand, ct, h2_of<R>(meta, i2),
                                       store + static_cast<size_t>(i2) * sv.ld, sv.copy1, row_bytes,
                                       SCALED ? scale[i2] : 1.0f);
        }
        if (i < i1)
            accum_trace<DT, W, SCALED>(acc, cand, ct, h2_of<R>(meta, i),
                                       store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes,
                                       SCALED ? scale[i] : 1.0f);
    }
}

template <int DT, int W, typename R>
__device__ __forceinline__ void accumulate_range(const StoreView &sv, const Cand<R> &cand, int32_t c_lo,
                                                 int32_t c_hi, int32_t first, int32_t step,
                                                 Acc<W, R> &acc)
{
    if (sv.scale)
        accumulate_cmps<DT, W, true, R>(sv, cand, c_lo, c_hi, first, step, acc);
    else
        accumulate_cmps<DT, W, false, R>(sv, cand, c_lo, c_hi, first, step, acc);
}

// ---------------------------------------------------------------------------
// candidate-batch semblance (lane = candidate)

template <int OP, int DT, int W, typename R>
__global__ __launch_bounds__(256) void k_eval(StoreView sv, CandView cv, R *__restrict__ S_out,
                                              int32_t *__restrict__ M_out)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = c < cv.n;
    const int64_t cc = live ? c : cv.n - 1;
    const int32_t j = cv.cmp[cc], n0 = cv.t[cc];
    const int32_t ap = sv.ap_tab[n0];
    R p[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int d = 0; d < OP; ++d) p[d] = static_cast<R>(cv.params[cc * OP + d]);
    const Cand<R> cand = make_cand<OP, R>(p, n0, j, ap, sv.nt, static_cast<R>(sv.dt),
                                          static_cast<R>(sv.dx));
    int32_t c_lo, c_hi;
    wave_cmp_range(sv, j, ap, live, c_lo, c_hi);
    Acc<W, R> acc;
    acc.reset();
    accumulate_range<DT, W, R>(sv, cand, c_lo, c_hi, 0, 1, acc);
    if (live) {
        S_out[c] = finish_semblance(acc);
        if (M_out) M_out[c] = acc.M;
    }
}

// Binary64 semblance of every grid sample's parameters (re-scoring).
template <int OP, int W>
__global__ __launch_bounds__(256) void k_eval64_grid(StoreView sv, const int32_t *__restrict__ cmp_out,
                                                     int32_t n_out, int32_t t_begin, int32_t n_t,
                                                     const float *__restrict__ params,
                                                     double *__restrict__ S_out)
{
    const int64_t total = static_cast<int64_t>(n_out) * n_t;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = c < total;
    const int64_t cc = live ? c : total - 1;
    const int32_t o = static_cast<int32_t>(cc / n_t);
    const int32_t n0 = t_begin + static_cast<int32_t>(cc - static_cast<int64_t>(o) * n_t);
    const int32_t j = cmp_out[o];
    const int32_t ap = sv.ap_tab[n0];
    double p[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < OP; ++d) p[d] = static_cast<double>(params[cc * OP + d]);
    const Cand<double> cand = make_cand<OP, double>(p, n0, j, ap, sv.nt, static_cast<double>(sv.dt),
                                                    static_cast<double>(sv.dx));
    int32_t c_lo, c_hi;
    wave_cmp_range(sv, j, ap, live, c_lo, c_hi);
    Acc<W, double> acc;
    acc.reset();
    accumulate_range<DT_F32, W, double>(sv, cand, c_lo, c_hi, 0, 1, acc);
    if (live) S_out[c] = finish_semblance(acc);
}

// ---------------------------------------------------------------------------
// adjoint: dS/dp through the interpolated gather, M held fixed.
//   dS/da_ik = 2/(M E) (s_k - M S a_ik),  da_ik/dtau = u[n+k+1] - u[n+k],
//   dtau/dp = (dq/dp) / (2 tau) with q in samples^2:
//   CMP q = n0^2 + C h^2/dt^2;  CRS q = (n0 + A dm/dt)^2 + B n0 dm^2/dt + C n0 h^2/dt.

template <int OP, int DT, int W>
__device__ __forceinline__ float semblance_grad_lane(const StoreView &sv, const Cand<float> &cand,
                                                     int32_t c_lo, int32_t c_hi, float *g)
{
    using T = typename Store<DT>::T;
    const T *store = static_cast<const T *>(sv.store);
    Acc<W, float> acc;
    acc.reset();
    accumulate_range<DT, W, float>(sv, cand, c_lo, c_hi, 0, 1, acc);
    const float S = finish_semblance(acc);
#pragma unroll
    for (int d = 0; d < OP; ++d) g[d] = 0.0f;
    const bool nonzero = acc.M > 0 && acc.E > 0.0f;
    const float coef = nonzero ? 2.0f / (static_cast<float>(acc.M) * acc.E) : 0.0f;
    const float MS = static_cast<float>(acc.M) * S;
    const float inv_dt = 1.0f / sv.dt;
    const ENS_CONST_AS int64_t *cmp_ptr = const_view(sv.cmp_ptr);
    const ENS_CONST_AS TraceMeta *meta = const_view(sv.meta);
    const ENS_CONST_AS float *scale = const_view(sv.scale);
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const CmpTerm<float> ct = cmp_term(cand, c, sv.dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
        for (int32_t i = static_cast<int32_t>(cmp_ptr[c]); i < i1; ++i) {
            const float h2 = meta[i].h2;
            const TT<float> tt = traveltime<W, sizeof(T)>(cand, ct, h2);
            const bool use = nonzero && tt.ok && tt.tau > 0.0f;
            const float sc = scale ? scale[i] : 1.0f;
            float u[W + 1];
            load_window<DT, W + 1>(store + static_cast<size_t>(i) * sv.ld, tt.off, sv.copy1,
                                   static_cast<uint32_t>(sv.ld * static_cast<int64_t>(sizeof(T))), u);
            const float wa = (1.0f - tt.f) * sc, wb = tt.f * sc;
            float dSdtau = 0.0f;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const float a = __builtin_fmaf(wb, u[k + 1], wa * u[k]);
                dSdtau = __builtin_fmaf(acc.s[k] - MS * a, (u[k + 1] - u[k]) * sc, dSdtau);
            }
            const float r = use ? coef * dSdtau / (2.0f * tt.tau) : 0.0f;
            if constexpr (OP == 1) {
                g[0] += r * h2 * inv_dt * inv_dt;
            } else {
                const float dm = ct.dm;
                g[0] += r * 2.0f * (cand.n0f + cand.As * dm) * dm * inv_dt;
                g[1] += r * cand.n0f * dm * dm * inv_dt;
                g[2] += r * cand.n0f * h2 * inv_dt;
            }
        }
    }
    return S;
}

template <int OP, int DT, int W>
__global__ __launch_bounds__(256) void k_backward(StoreView sv, CandView cv, const float *__restrict__ dS,
                                                  float *__restrict__ g_out)
{
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = c < cv.n;
    const int64_t cc = live ? c : cv.n - 1;
    const int32_t j = cv.cmp[cc], n0 = cv.t[cc];
    const int32_t ap = sv.ap_tab[n0];
    float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < OP; ++d) p[d] = cv.params[cc * OP + d];
    const Cand<float> cand = make_cand<OP, float>(p, n0, j, ap, sv.nt, sv.dt, sv.dx);
    int32_t c_lo, c_hi;
    wave_cmp_range(sv, j, ap, live, c_lo, c_hi);
    float g[3];
    semblance_grad_lane<OP, DT, W>(sv, cand, c_lo, c_hi, g);
    if (live) {
        const float ds = dS[c];
#pragma unroll
        for (int d = 0; d < OP; ++d) g_out[c * OP + d] = ds * g[d];
    }
}

// ---------------------------------------------------------------------------
// evolution

// Best member of the population occupying lanes [base, base+np): highest
// score, lowest slot on ties (section "Sorting" with P = 1).
__device__ __forceinline__ int32_t group_argmax(float S, int32_t base, int32_t np)
{
    float best = __shfl(S, base, WAVE);
    int32_t bi = 0;
    for (int32_t q = 1; q < np; ++q) {
        const float v = __shfl(S, base + q, WAVE);
        if (v > best) {
            best = v;
            bi = q;
        }
    }
    return bi;
}

// Trial vector of this lane's slot: current-to-best/1 mutant from the slot,
// the best and two other random members, binomial crossover (section
// "Mutation and crossover").  Every lane of the wave must call it.
// With an archive (JADE), lane base + a holds archive entry a in `arch`
// and r2 ranges over the np members and the n_arch entries.
template <int P, bool ARCHIVE = false>
__device__ __forceinline__ void make_trial(const float *x, float S, int32_t base, int32_t np,
                                          int32_t slot, const uint64_t w[4], float F, uint64_t cr_thr,
                                          const float *lo, const float *hi, float *u,
                                          const float *arch = nullptr, int32_t n_arch = 0)
{
    const int32_t b = group_argmax(S, base, np);
    const TrialDraw dr = trial_draw(w, slot, np, P, cr_thr, ARCHIVE ? np + n_arch : np);
    const bool from_arch = ARCHIVE && dr.r2 >= static_cast<uint32_t>(np);
    const int32_t r2_lane = base + static_cast<int32_t>(from_arch ? dr.r2 - np : dr.r2);
#pragma unroll
    for (int d = 0; d < P; ++d) {
        const float xb = __shfl(x[d], base + b, WAVE);
        const float xr1 = __shfl(x[d], base + static_cast<int32_t>(dr.r1), WAVE);
        float xr2 = __shfl(x[d], r2_lane, WAVE);
        if constexpr (ARCHIVE) {
            const float ar2 = __shfl(arch[d], r2_lane, WAVE);
            xr2 = from_arch ? ar2 : xr2;
        }
        const float v = mutant(x[d], xb, xr1, xr2, F, lo[d], hi[d]);
        u[d] = dr.take[d] ? v : x[d];
    }
}

// JADE bookkeeping after a generation's evaluation, in slot order within
// each population: every slot whose trial replaces its parent (ok) puts the
// parent into the archive (appended while it holds fewer than np entries,
// else at that slot's drawn position) and adds its F and CR to the
// population's sums; then the means move toward the successful values.
// Every lane of the wave must call it; populations are lane groups.
template <int P>
__device__ __forceinline__ void jade_update(bool ok, const float *x, int32_t k_cr, int32_t k_f, int32_t a_idx,
                                           int32_t grp, int32_t np, int32_t slot, float *arch, int32_t &n_arch,
                                           double &mu_cr, double &mu_f)
{
    uint64_t pending = __ballot(ok);
    int64_t s_cr = 0, s_f = 0, s_f2 = 0;
    int32_t n_s = 0;
    while (pending) {
        const int32_t L = __builtin_ctzll(pending);
        pending &= pending - 1;
        float xs[3];
#pragma unroll
        for (int d = 0; d < P; ++d) xs[d] = __shfl(x[d], L, WAVE);
        const int32_t kc = __shfl(k_cr, L, WAVE), kf = __shfl(k_f, L, WAVE), ai = __shfl(a_idx, L, WAVE);
        if (L / np == grp) {
            const int32_t pos = n_arch < np ? n_arch : ai;
            if (slot == pos) {
#pragma unroll
                for (int d = 0; d < P; ++d) arch[d] = xs[d];
            }
            n_arch = n_arch < np ? n_arch + 1 : np;
            n_s += 1;
            s_cr += kc;
            s_f += kf;
            s_f2 += static_cast<int64_t>(kf) * kf;
        }
    }
    if (n_s > 0) {
        const double mean_cr = static_cast<double>(s_cr) / (static_cast<double>(n_s) * JADE_GRID);
        const double lehmer_f = static_cast<double>(s_f2) / (static_cast<double>(s_f) * JADE_GRID);
        mu_cr = 0.9 * mu_cr + 0.1 * mean_cr;
        mu_f = 0.9 * mu_f + 0.1 * lehmer_f;
    }
}

template <int P>
__device__ __forceinline__ void load_clamped(const float *__restrict__ src, const float *lo,
                                             const float *hi, float *x)
{
#pragma unroll
    for (int d = 0; d < P; ++d) {
        float v = src[d];
        v = v < lo[d] ? lo[d] : v;
        v = v > hi[d] ? hi[d] : v;
        x[d] = v;
    }
}

// Semblance of each lane's candidate, the trace loop split over the
// workgroup's nsl waves (in every CMP, wave w takes the CMP's traces w,
// w + nsl, w + 2 nsl, ...);
// partial sums meet in LDS and every wave adds them in the same order.
template <int DT, int W>
__device__ __forceinline__ float eval_slices(const StoreView &sv, const Cand<float> &cand, int32_t c_lo,
                                             int32_t c_hi, int32_t wave, int32_t nsl, int32_t lane,
                                             float *lds, int &buf, int32_t &M)
{
    Acc<W, float> acc;
    acc.reset();
    accumulate_range<DT, W, float>(sv, cand, c_lo, c_hi, wave, nsl, acc);
    if (nsl > 1) {
        float *mine = lds + ((buf * nsl + wave) * (W + 2)) * WAVE + lane;
#pragma unroll
        for (int k = 0; k < W; ++k) mine[k * WAVE] = acc.s[k];
        mine[W * WAVE] = acc.E;
        mine[(W + 1) * WAVE] = __int_as_float(acc.M);
        __syncthreads();
        acc.reset();
        for (int32_t v = 0; v < nsl; ++v) {
            const float *r = lds + ((buf * nsl + v) * (W + 2)) * WAVE + lane;
#pragma unroll
            for (int k = 0; k < W; ++k) acc.s[k] += r[k * WAVE];
            acc.E += r[W * WAVE];
            acc.M += __float_as_int(r[(W + 1) * WAVE]);
        }
        buf ^= 1;
    }
    M = acc.M;
    return finish_semblance(acc);
}

// Evolution of a group of samples: lane = (sample, slot), floor(64/NP)
// samples of one output CMP per wave, the trace loop split over nsl waves.
// Sweep pacing.  Every workgroup of an ENS launch sweeps the same number of
// trace steps and all of them are resident together, so the launch lasts as
// long as its slowest sweep.  The wave arbiter favours older waves, which lets
// the first-dispatched sweeps race ahead and leaves the last ones to finish
// alone on a half-empty chip.  Before each step a wave compares its progress
// with the launch's mean (steps counts every finished step of every
// workgroup) and takes a high issue priority when behind, a low one when
// ahead; the results do not depend on it.
__device__ __forceinline__ void pace_by_progress(const unsigned long long *steps, int32_t done_here)
{
    const unsigned long long all = __hip_atomic_load(steps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t total = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(all)));
    const int64_t mine = static_cast<int64_t>(done_here) * gridDim.x;
    const int64_t half = gridDim.x / 2;
    if (mine + half < total)
        __builtin_amdgcn_s_setprio(3);
    else if (mine > total + half)
        __builtin_amdgcn_s_setprio(0);
    else
        __builtin_amdgcn_s_setprio(1);
}

// Plain search: each workgroup runs the whole evolution (initial population
// and NG generations) of its samples.  ENS: each workgroup sweeps its time
// samples through the traces of its bucket, one trace after another: within
// a stage, sample (t, trace) depends only on (t, previous trace) of the same
// stage and on the complete previous stage, so the sweeps of different t
// never wait for each other and one launch covers many steps.
// KIND 0: exploration (plain evolution or ENS stage 0); KIND 1: ENS
// exploitation stages.  KIND selects the counters and names the kernel.
// k_search_dense is the same code held to 64 VGPRs (8 waves per SIMD), for
// launches whose wave count fits the chip in one round at that occupancy.
template <int OP, int DT, int W, int KIND, bool ADAPT>
__device__ __forceinline__ void search_body(const SearchArgs &a)
{
    extern __shared__ float lds[];
    const int32_t nsl = a.nsl;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(threadIdx.x) >> 6);
    const int32_t lane = threadIdx.x & (WAVE - 1);
    const int4 it = a.items[a.xcd_order ? xcd_remap(blockIdx.x, gridDim.x) : static_cast<int32_t>(blockIdx.x)];
    // the traces this workgroup sweeps: one for the plain search, else the
    // steps [k_begin, k_end) of its bucket's sweep (fewer for a short bucket)
    int32_t b0 = 0, nb = 1, k_end = 1, k_begin = 0;
    if (!a.plain) {
        b0 = it.x * a.n_bucket;
        nb = min(a.n_bucket, a.n_out - b0);
        k_begin = a.k_begin;
        k_end = min(a.k_end, nb);
    }
    // item: t_start, ns samples t_start + m stride (stride in bits 8..15), NP
    const int32_t t_start = it.y, ns = it.z & 0xff, stride = it.z >> 8, np = it.w;
    const int32_t grp = lane / np;
    const bool live = grp < ns;
    const int32_t slot = lane - grp * np;
    const int32_t base = grp * np;
    const int32_t n0 = t_start + (live ? grp : ns - 1) * stride;
    const int32_t tt = n0 - a.t_begin;
    const int32_t ap = a.sv.ap_tab[n0];
    float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < OP; ++d) {
        lo[d] = a.lo_tab[n0 * 3 + d];
        hi[d] = a.hi_tab[n0 * 3 + d];
    }
    // apertures grow or shrink linearly in t: the item's extreme samples bound them
    const int32_t amax = max(a.sv.ap_tab[t_start], a.sv.ap_tab[t_start + (ns - 1) * stride]);
    const uint64_t stage = static_cast<uint64_t>(a.stage);
    int buf = 0;
    int32_t M = 0;
    uint32_t n_ev = 0;
    uint64_t sum_m = 0;
    float pbest[3] = {0.f, 0.f, 0.f};  // this sample's best on the previous trace of the sweep

    for (int32_t k = k_begin; k < k_end; ++k) {
        if (a.progress) pace_by_progress(a.progress, k - k_begin);
        const int32_t o = a.plain ? it.x : b0 + (a.forward ? k : nb - 1 - k);
        const int32_t prev = k > 0 ? (a.forward ? o - 1 : o + 1) : -1;
        const int32_t j = __builtin_amdgcn_readfirstlane(a.cmp_out[o]);
        const int32_t c_lo = max(0, j - amax), c_hi = min(a.sv.n_cmp - 1, j + amax);
        const uint64_t sid =
            static_cast<uint64_t>(n0) + static_cast<uint64_t>(a.sv.nt) * static_cast<uint64_t>(j);
        const int64_t here = static_cast<int64_t>(o) * a.n_t + tt;

        // initial population (section "Initializing") and ENS seeds
        float x[3] = {0.f, 0.f, 0.f};
        uint64_t w[4];
        philox4x64_10(sid, stage, 0, static_cast<uint64_t>(slot), a.seed, 0, w);
#pragma unroll
        for (int d = 0; d < OP; ++d) x[d] = init_coord(w[d], lo[d], hi[d]);
        float S = 0.0f;
        bool scored = false;
        if (!a.plain) {
            // the previous trace of this sweep: kept in registers within the
            // launch, read back from the stage state at a launch's first step
            const int prev_slot = a.stage == 0 ? 0 : 2;
            if (a.inject && slot == prev_slot && prev >= 0) {
                if (k > k_begin) {
#pragma unroll
                    for (int d = 0; d < OP; ++d) x[d] = fminf(fmaxf(pbest[d], lo[d]), hi[d]);
                } else {
                    load_clamped<OP>(a.Yp + (static_cast<int64_t>(prev) * a.n_t + tt) * OP, lo, hi, x);
                }
            }
            if (a.stage > 0) {
                if (a.inject && slot == 0 && tt > 0) load_clamped<OP>(a.Xp + (here - 1) * OP, lo, hi, x);
                if (a.inject && slot == 1 && tt < a.n_t - 1)
                    load_clamped<OP>(a.Xp + (here + 1) * OP, lo, hi, x);
                if (slot == 3) {
#pragma unroll
                    for (int d = 0; d < OP; ++d) x[d] = a.Xp[here * OP + d];
                    S = a.XS[here];
                    scored = true;
                }
            }
        }
        {
            const Cand<float> cand = make_cand<OP, float>(x, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            const float Sev = eval_slices<DT, W>(a.sv, cand, c_lo, c_hi, wave, nsl, lane, lds, buf, M);
            if (!scored) {
                S = Sev;
                if (live) {
                    n_ev += 1;
                    sum_m += static_cast<uint64_t>(M);
                }
            }
        }
        // generations (sections "Mutation and crossover", "Selection"); with
        // ADAPT, JADE's control parameters and archive, reset per domain
        double mu_cr = static_cast<double>(a.CR), mu_f = static_cast<double>(a.F);
        int32_t n_arch = 0;
        float arch[3] = {0.f, 0.f, 0.f};
        for (int32_t g = 1; g <= a.ng; ++g) {
            philox4x64_10(sid, stage, static_cast<uint64_t>(g), static_cast<uint64_t>(slot), a.seed, 0,
                          w);
            float u[3] = {0.f, 0.f, 0.f};
            int32_t k_cr = 0, k_f = 0, a_idx = 0;
            if constexpr (ADAPT) {
                uint64_t jw[4];
                philox4x64_10(sid, stage + (1ULL << 32), static_cast<uint64_t>(g), static_cast<uint64_t>(slot),
                              a.seed, 0, jw);
                jade_draws(jw, mu_cr, mu_f, np, k_cr, k_f, a_idx);
                const float F = static_cast<float>(k_f) * 0x1p-24f;
                make_trial<OP, true>(x, S, base, np, slot, w, F, static_cast<uint64_t>(k_cr) << 8, lo, hi, u,
                                     arch, n_arch);
            } else {
                make_trial<OP>(x, S, base, np, slot, w, a.F, a.cr_thr, lo, hi, u);
            }
            const Cand<float> cand = make_cand<OP, float>(u, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            const float St = eval_slices<DT, W>(a.sv, cand, c_lo, c_hi, wave, nsl, lane, lds, buf, M);
            if (live) {
                n_ev += 1;
                sum_m += static_cast<uint64_t>(M);
            }
            if constexpr (ADAPT)
                jade_update<OP>(St >= S, x, k_cr, k_f, a_idx, grp, np, slot, arch, n_arch, mu_cr, mu_f);
            if (St >= S) {
#pragma unroll
                for (int d = 0; d < OP; ++d) x[d] = u[d];
                S = St;
            }
        }
        const int32_t b = group_argmax(S, base, np);
#pragma unroll
        for (int d = 0; d < OP; ++d) pbest[d] = __shfl(x[d], base + b, WAVE);
        if (wave == 0 && live && slot == b) {
#pragma unroll
            for (int d = 0; d < OP; ++d) a.Yp[here * OP + d] = x[d];
            a.YS[here] = S;
        }
        if (a.progress && threadIdx.x == 0) atomicAdd(a.progress, 1ull);
    }
    if (wave == 0) {
        const uint64_t tot_ev = wave_sum(static_cast<uint64_t>(n_ev));
        const uint64_t tot_m = wave_sum(sum_m);
        if (lane == 0) {
            atomicAdd(a.counters + 2 * KIND, static_cast<unsigned long long>(tot_ev));
            atomicAdd(a.counters + 2 * KIND + 1, static_cast<unsigned long long>(tot_m));
        }
    }
}

// Time-sample skipping: after a stage, every sample it did not estimate
// takes the parameters interpolated linearly in t between the nearest
// estimated samples of the stage on the same trace (the nearest one alone at
// the grid ends), clamped into its box, and is scored once; from the second
// stage on the interpolated individual replaces the stored one only when it
// scores higher (section "The performance-quality trade-off by an
// interpolation process").  Lane = (output CMP, time sample).
template <int OP, int DT, int W>
__global__ __launch_bounds__(256) void k_interp(InterpArgs a)
{
    const int64_t total = static_cast<int64_t>(a.n_out) * a.n_t;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in_grid = c < total;
    const int64_t cc = in_grid ? c : total - 1;
    const int32_t o = static_cast<int32_t>(cc / a.n_t);
    const int32_t tt = static_cast<int32_t>(cc - static_cast<int64_t>(o) * a.n_t);
    const int32_t stride = a.stride, init = a.init;
    const bool estimated = tt >= init && (tt - init) % stride == 0;
    const int32_t ta = tt > init ? tt - (tt - init) % stride : -1;
    const int32_t tb_ = tt < init ? init : tt - (tt - init) % stride + stride;
    const int32_t tb = tb_ < a.n_t ? tb_ : -1;
    const bool has = ta >= 0 || tb >= 0;
    const bool live = in_grid && !estimated;
    const int32_t n0 = a.t_begin + tt;
    const int32_t j = a.cmp_out[o];
    const int32_t ap = a.sv.ap_tab[n0];
    const int64_t row = static_cast<int64_t>(o) * a.n_t;
    float p[3] = {0.f, 0.f, 0.f};
    if (has) {
        const float *pa = a.Yp + (row + (ta >= 0 ? ta : tb)) * OP;
        const float *pb = a.Yp + (row + (tb >= 0 ? tb : ta)) * OP;
        if (ta >= 0 && tb >= 0) {
            const float wgt = static_cast<float>(tt - ta) / static_cast<float>(tb - ta);
#pragma unroll
            for (int d = 0; d < OP; ++d) {
                const float diff = pb[d] - pa[d];
                const float step = wgt * diff;
                p[d] = pa[d] + step;
            }
        } else {
#pragma unroll
            for (int d = 0; d < OP; ++d) p[d] = pa[d];
        }
#pragma unroll
        for (int d = 0; d < OP; ++d) {
            p[d] = fmaxf(p[d], a.lo_tab[n0 * 3 + d]);
            p[d] = fminf(p[d], a.hi_tab[n0 * 3 + d]);
        }
    }
    const Cand<float> cand = make_cand<OP, float>(p, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
    int32_t c_lo, c_hi;
    wave_cmp_range(a.sv, j, ap, live && has, c_lo, c_hi);
    Acc<W, float> acc;
    acc.reset();
    accumulate_range<DT, W, float>(a.sv, cand, c_lo, c_hi, 0, 1, acc);
    const float Sp = finish_semblance(acc);
    const bool counted = live && has;
    if (live) {
        const int64_t here = row + tt;
        if (has && (a.stage == 0 || Sp > a.XS[here])) {
#pragma unroll
            for (int d = 0; d < OP; ++d) a.Yp[here * OP + d] = p[d];
            a.YS[here] = Sp;
        } else if (a.stage > 0) {
#pragma unroll
            for (int d = 0; d < OP; ++d) a.Yp[here * OP + d] = a.Xp[here * OP + d];
            a.YS[here] = a.XS[here];
        }
    }
    const uint64_t n = wave_sum(static_cast<uint64_t>(counted ? 1 : 0));
    const uint64_t m = wave_sum(static_cast<uint64_t>(counted ? acc.M : 0));
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        atomicAdd(a.counters + 2 * a.kind, static_cast<unsigned long long>(n));
        atomicAdd(a.counters + 2 * a.kind + 1, static_cast<unsigned long long>(m));
    }
}

// Zero-offset stack of every grid sample along its operator: the mean over
// the participating traces of the amplitude interpolated at the traveltime
// (0 for an empty fold), from the binary32 copy of the traces (sections
// "Traveltime parameter search", "Qualitative analysis").  Lane = sample.
template <int OP>
__global__ __launch_bounds__(256) void k_stack(StoreView sv, const int32_t *__restrict__ cmp_out, int32_t n_out,
                                               int32_t t_begin, int32_t n_t, const float *__restrict__ params,
                                               float *__restrict__ out)
{
    const int64_t total = static_cast<int64_t>(n_out) * n_t;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = c < total;
    const int64_t cc = live ? c : total - 1;
    const int32_t o = static_cast<int32_t>(cc / n_t);
    const int32_t n0 = t_begin + static_cast<int32_t>(cc - static_cast<int64_t>(o) * n_t);
    const int32_t j = cmp_out[o];
    const int32_t ap = sv.ap_tab[n0];
    float p[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < OP; ++d) p[d] = params[cc * OP + d];
    const Cand<float> cand = make_cand<OP, float>(p, n0, j, ap, sv.nt, sv.dt, sv.dx);
    int32_t c_lo, c_hi;
    wave_cmp_range(sv, j, ap, live, c_lo, c_hi);
    const float *store = static_cast<const float *>(sv.store);
    const ENS_CONST_AS int64_t *cmp_ptr = const_view(sv.cmp_ptr);
    const ENS_CONST_AS TraceMeta *meta = const_view(sv.meta);
    float sum = 0.0f;
    int32_t M = 0;
    for (int32_t cm = c_lo; cm <= c_hi; ++cm) {
        const CmpTerm<float> ct = cmp_term(cand, cm, sv.dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[cm + 1]);
        for (int32_t i = static_cast<int32_t>(cmp_ptr[cm]); i < i1; ++i) {
            // a one-sample window: off is the byte offset of the sample before the traveltime
            const TT<float> tt = traveltime<1, 4>(cand, ct, meta[i].h2);
            const float *row = store + static_cast<size_t>(i) * sv.ld;
            const float *p0 = reinterpret_cast<const float *>(reinterpret_cast<const char *>(row) + tt.off);
            const float u0 = p0[0], u1 = p0[1];
            sum += fmadd(tt.f, u1, (1.0f - tt.f) * u0);
            M += tt.ok ? 1 : 0;
        }
    }
    if (live) out[c] = M > 0 ? sum / static_cast<float>(M) : 0.0f;
}

// Root mean square of a panel in binary64, one workgroup, fixed summation
// order (section "Quantitative analysis": methods compared by the RMS of
// their coherence panels).
__global__ __launch_bounds__(1024) void k_rms(const float *__restrict__ x, int64_t n, double *__restrict__ out)
{
    __shared__ double part[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double v = static_cast<double>(x[i]);
        s = __builtin_fma(v, v, s);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? __builtin_sqrt(part[0] / static_cast<double>(n)) : 0.0;
}

template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) void k_search(SearchArgs a)
{
    search_body<OP, DT, W, KIND, false>(a);
}

template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_search_dense(SearchArgs a)
{
    search_body<OP, DT, W, KIND, false>(a);
}

// the same search with JADE's control-parameter adaptation and archive
template <int OP, int DT, int W, int KIND>
__global__ __launch_bounds__(512) void k_search_jade(SearchArgs a)
{
    search_body<OP, DT, W, KIND, true>(a);
}

// Gradient polish of each grid sample's winner: Adam (beta1 0.9, beta2 0.999,
// eps 1e-8) ascending S on box-normalised coordinates, projected onto the
// box, scoring every step and keeping the best point (lane = sample).
template <int OP, int DT, int W>
__global__ __launch_bounds__(256) void k_polish(PolishArgs a)
{
    const int64_t total = static_cast<int64_t>(a.n_out) * a.n_t;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool live = c < total;
    const int64_t cc = live ? c : total - 1;
    const int32_t o = static_cast<int32_t>(cc / a.n_t);
    const int32_t n0 = a.t_begin + static_cast<int32_t>(cc - static_cast<int64_t>(o) * a.n_t);
    const int32_t j = a.cmp_out[o];
    const int32_t ap = a.sv.ap_tab[n0];
    float lo[3] = {0.f, 0.f, 0.f}, span[3] = {1.f, 1.f, 1.f}, p[3] = {0.f, 0.f, 0.f};
    float z[3], m[3] = {0.f, 0.f, 0.f}, v[3] = {0.f, 0.f, 0.f}, best[3];
#pragma unroll
    for (int d = 0; d < OP; ++d) {
        lo[d] = a.lo_tab[n0 * 3 + d];
        span[d] = a.hi_tab[n0 * 3 + d] - lo[d];
        p[d] = a.params[cc * OP + d];
        best[d] = p[d];
        z[d] = (p[d] - lo[d]) / span[d];
    }
    float best_S = a.S[cc];
    if (live && a.S_pre) a.S_pre[c] = best_S;
    int32_t c_lo, c_hi;
    wave_cmp_range(a.sv, j, ap, live, c_lo, c_hi);
    float b1k = 1.0f, b2k = 1.0f;
    uint64_t sum_m = 0;
    for (int32_t k = 1; k <= a.steps; ++k) {
        float g[3];
        {
            const Cand<float> cand = make_cand<OP, float>(p, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
            semblance_grad_lane<OP, DT, W>(a.sv, cand, c_lo, c_hi, g);
        }
        b1k *= 0.9f;
        b2k *= 0.999f;
#pragma unroll
        for (int d = 0; d < OP; ++d) {
            const float gz = g[d] * span[d];
            m[d] = 0.9f * m[d] + 0.1f * gz;
            v[d] = 0.999f * v[d] + 0.001f * gz * gz;
            const float mh = m[d] / (1.0f - b1k), vh = v[d] / (1.0f - b2k);
            z[d] += a.lr * mh / (__builtin_sqrtf(vh) + 1e-8f);
            z[d] = fminf(fmaxf(z[d], 0.0f), 1.0f);
            p[d] = lo[d] + z[d] * span[d];
        }
        const Cand<float> cand = make_cand<OP, float>(p, n0, j, ap, a.sv.nt, a.sv.dt, a.sv.dx);
        Acc<W, float> acc;
        acc.reset();
        accumulate_range<DT, W, float>(a.sv, cand, c_lo, c_hi, 0, 1, acc);
        const float Sn = finish_semblance(acc);
        sum_m += live ? static_cast<uint64_t>(acc.M) : 0;
        if (Sn > best_S) {
            best_S = Sn;
#pragma unroll
            for (int d = 0; d < OP; ++d) best[d] = p[d];
        }
    }
    if (live) {
#pragma unroll
        for (int d = 0; d < OP; ++d) a.params[c * OP + d] = best[d];
        a.S[c] = best_S;
    }
    const uint64_t n = wave_sum(static_cast<uint64_t>(live ? a.steps : 0));
    const uint64_t msum = wave_sum(sum_m);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        atomicAdd(a.counters + 4, static_cast<unsigned long long>(n));
        atomicAdd(a.counters + 5, static_cast<unsigned long long>(msum));
    }
}

// ---------------------------------------------------------------------------
// building-block checks

__global__ void k_philox(int64_t n, const uint64_t *__restrict__ ctr, const uint64_t *__restrict__ key,
                         uint64_t *__restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t w[4];
    philox4x64_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[0], key[1], w);
#pragma unroll
    for (int k = 0; k < 4; ++k) out[4 * i + k] = w[k];
}

// One population per wave, lane = slot.
template <int P>
__global__ __launch_bounds__(64) void k_de_trial(int32_t np, const float *__restrict__ pop,
                                                 const float *__restrict__ S,
                                                 const uint64_t *__restrict__ words, float F,
                                                 uint64_t cr_thr, const float *__restrict__ lo_in,
                                                 const float *__restrict__ hi_in,
                                                 float *__restrict__ trial)
{
    const int32_t pi = blockIdx.x;
    const int32_t lane = threadIdx.x;
    const bool live = lane < np;
    const int32_t slot = live ? lane : np - 1;
    const int64_t row = static_cast<int64_t>(pi) * np + slot;
    float x[3] = {0.f, 0.f, 0.f}, lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f}, u[3];
#pragma unroll
    for (int d = 0; d < P; ++d) {
        x[d] = pop[row * P + d];
        lo[d] = lo_in[pi * P + d];
        hi[d] = hi_in[pi * P + d];
    }
    uint64_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = words[row * 4 + k];
    make_trial<P>(x, S[row], 0, np, slot, w, F, cr_thr, lo, hi, u);
    if (live) {
#pragma unroll
        for (int d = 0; d < P; ++d) trial[row * P + d] = u[d];
    }
}

// JADE's per-slot draws for n generator blocks (a check of the device routine).
__global__ __launch_bounds__(256) void k_jade_draws(int64_t n, const uint64_t *__restrict__ words, double mu_cr,
                                                    double mu_f, int32_t np, int32_t *__restrict__ k_cr,
                                                    int32_t *__restrict__ k_f, int32_t *__restrict__ a_idx)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = words[i * 4 + k];
    int32_t c, f, a;
    jade_draws(w, mu_cr, mu_f, np, c, f, a);
    k_cr[i] = c;
    k_f[i] = f;
    a_idx[i] = a;
}

// ---------------------------------------------------------------------------
// launch wrappers

bool window_supported(int window)
{
    return window == 3 || window == 5 || window == 7 || window == 9 || window == 11 ||
           window == 13 || window == 15;
}

#define ENS_DISPATCH_W(window, ...)                        \
    switch (window) {                                      \
    case 3: { constexpr int W = 3; __VA_ARGS__; } break;   \
    case 5: { constexpr int W = 5; __VA_ARGS__; } break;   \
    case 7: { constexpr int W = 7; __VA_ARGS__; } break;   \
    case 9: { constexpr int W = 9; __VA_ARGS__; } break;   \
    case 11: { constexpr int W = 11; __VA_ARGS__; } break; \
    case 13: { constexpr int W = 13; __VA_ARGS__; } break; \
    case 15: { constexpr int W = 15; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                  \
    }

#define ENS_DISPATCH_OP(op, ...)                           \
    if ((op) == 1) { constexpr int OP = 1; __VA_ARGS__; }  \
    else { constexpr int OP = 3; __VA_ARGS__; }

#define ENS_DISPATCH_DT(dt, ...)                                           \
    switch (dt) {                                                          \
    case DT_F32: { constexpr int DT = DT_F32; __VA_ARGS__; } break;        \
    case DT_F16: { constexpr int DT = DT_F16; __VA_ARGS__; } break;        \
    case DT_BF16: { constexpr int DT = DT_BF16; __VA_ARGS__; } break;      \
    default: return hipErrorInvalidValue;                                  \
    }

static inline unsigned blocks_for(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

hipError_t launch_store_f32(const float *src, int64_t ld_in, int64_t n_tr, int32_t nt, int64_t ld,
                            float *dst, hipStream_t s)
{
    if (n_tr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_f32, dim3(static_cast<unsigned>(n_tr)), dim3(256), 0, s, src, ld_in,
                       nt, ld, dst);
    return hipGetLastError();
}

hipError_t launch_quantize(const float *src, int64_t ld_in, int64_t n_tr, int32_t nt, int32_t dtype,
                           uint16_t *dst, int64_t ld_out, int32_t col0, float *scale, bool dual, hipStream_t s)
{
    if (n_tr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_quantize, dim3(static_cast<unsigned>(n_tr)), dim3(256), 0, s, src, ld_in, nt,
                       dtype, dst, ld_out, col0, scale, static_cast<int32_t>(dual));
    return hipGetLastError();
}

hipError_t launch_eval(int op, int dtype, int window, const StoreView &sv, const CandView &cv,
                       float *S, int32_t *M, hipStream_t s)
{
    if (cv.n == 0) return hipSuccess;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_eval<OP, DT, W, float>), dim3(blocks_for(cv.n, 256)), dim3(256), 0, s,
                           sv, cv, S, M))));
    return hipGetLastError();
}

hipError_t launch_eval64(int op, int window, const StoreView &sv, const CandView &cv, double *S,
                         hipStream_t s)
{
    if (cv.n == 0) return hipSuccess;
    int32_t *no_M = nullptr;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_eval<OP, DT_F32, W, double>), dim3(blocks_for(cv.n, 256)), dim3(256), 0,
                           s, sv, cv, S, no_M)));
    return hipGetLastError();
}

hipError_t launch_eval64_grid(int op, int window, const StoreView &sv, const int32_t *cmp_out,
                              int32_t n_out, int32_t t_begin, int32_t n_t, const float *params,
                              double *S, hipStream_t s)
{
    const int64_t total = static_cast<int64_t>(n_out) * n_t;
    if (total == 0) return hipSuccess;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_eval64_grid<OP, W>), dim3(blocks_for(total, 256)), dim3(256), 0, s, sv,
                           cmp_out, n_out, t_begin, n_t, params, S)));
    return hipGetLastError();
}

hipError_t launch_backward(int op, int dtype, int window, const StoreView &sv, const CandView &cv,
                           const float *dS, float *g, hipStream_t s)
{
    if (cv.n == 0) return hipSuccess;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_backward<OP, DT, W>), dim3(blocks_for(cv.n, 256)), dim3(256), 0, s, sv,
                           cv, dS, g))));
    return hipGetLastError();
}

hipError_t launch_search(int op, int dtype, int window, int kind, int dense, const SearchArgs &a,
                         int32_t n_blocks, hipStream_t s)
{
    if (n_blocks == 0) return hipSuccess;
    const size_t lds = a.nsl > 1 ? sizeof(float) * 2 * a.nsl * (window + 2) * WAVE : 0;
    const dim3 grid(static_cast<unsigned>(n_blocks)), block(WAVE * a.nsl);
    if (a.adapt && kind == 0) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_jade<OP, DT, W, 0>), grid, block, lds, s, a))));
    } else if (a.adapt) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_jade<OP, DT, W, 1>), grid, block, lds, s, a))));
    } else if (kind == 0 && !dense) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search<OP, DT, W, 0>), grid, block, lds, s, a))));
    } else if (kind == 0) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_dense<OP, DT, W, 0>), grid, block, lds, s, a))));
    } else if (!dense) {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search<OP, DT, W, 1>), grid, block, lds, s, a))));
    } else {
        ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
            hipLaunchKernelGGL((k_search_dense<OP, DT, W, 1>), grid, block, lds, s, a))));
    }
    return hipGetLastError();
}

hipError_t launch_stack(int op, const StoreView &sv_f32, const int32_t *cmp_out, int32_t n_out, int32_t t_begin,
                        int32_t n_t, const float *params, float *out, hipStream_t s)
{
    const int64_t total = static_cast<int64_t>(n_out) * n_t;
    if (total == 0) return hipSuccess;
    if (op == 1)
        hipLaunchKernelGGL(k_stack<1>, dim3(blocks_for(total, 256)), dim3(256), 0, s, sv_f32, cmp_out, n_out,
                           t_begin, n_t, params, out);
    else
        hipLaunchKernelGGL(k_stack<3>, dim3(blocks_for(total, 256)), dim3(256), 0, s, sv_f32, cmp_out, n_out,
                           t_begin, n_t, params, out);
    return hipGetLastError();
}

hipError_t launch_rms(const float *x, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_rms, dim3(1), dim3(1024), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_interp(int op, int dtype, int window, const InterpArgs &a, hipStream_t s)
{
    const int64_t total = static_cast<int64_t>(a.n_out) * a.n_t;
    if (total == 0) return hipSuccess;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_interp<OP, DT, W>), dim3(blocks_for(total, 256)), dim3(256), 0, s, a))));
    return hipGetLastError();
}

hipError_t launch_polish(int op, int dtype, int window, const PolishArgs &a, hipStream_t s)
{
    const int64_t total = static_cast<int64_t>(a.n_out) * a.n_t;
    if (total == 0 || a.steps <= 0) return hipSuccess;
    ENS_DISPATCH_OP(op, ENS_DISPATCH_DT(dtype, ENS_DISPATCH_W(window,
        hipLaunchKernelGGL((k_polish<OP, DT, W>), dim3(blocks_for(total, 256)), dim3(256), 0, s, a))));
    return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint64_t *ctr, const uint64_t *key, uint64_t *out,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, ctr, key, out);
    return hipGetLastError();
}

hipError_t launch_jade_draws(int64_t n, const uint64_t *words, double mu_cr, double mu_f, int32_t np,
                             int32_t *k_cr, int32_t *k_f, int32_t *a_idx, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jade_draws, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, words, mu_cr, mu_f, np, k_cr,
                       k_f, a_idx);
    return hipGetLastError();
}

hipError_t launch_de_trial(int32_t n_pop, int32_t np, int32_t P, const float *pop, const float *S,
                           const uint64_t *words, float F, uint64_t cr_thr, const float *lo,
                           const float *hi, float *trial, hipStream_t s)
{
    if (n_pop == 0) return hipSuccess;
    if (P == 1)
        hipLaunchKernelGGL(k_de_trial<1>, dim3(n_pop), dim3(64), 0, s, np, pop, S, words, F, cr_thr, lo,
                           hi, trial);
    else
        hipLaunchKernelGGL(k_de_trial<3>, dim3(n_pop), dim3(64), 0, s, np, pop, S, words, F, cr_thr, lo,
                           hi, trial);
    return hipGetLastError();
}

}  // namespace ens
