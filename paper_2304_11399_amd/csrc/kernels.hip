// HIP kernels of libens (gfx950) and their launch wrappers.
#include "search.h"

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

// One workgroup (256 threads) per trace: the scale is the smallest power of
// two at or above max|u| (1 when the trace is zero), q = RNE(u / scale), the
// quotient exact in binary32.  Output row stride ld_out with the first sample
// at column col0; when col0 > 0 the whole padded row is written.
// dual: the row is written twice, [0, ld_out) as laid out and
// [ld_out, 2 ld_out) shifted left by one sample (column c holds column c + 1).
// exp_out (optional): the scale's exponent, INT32_MIN for a zero trace.
__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ src, int64_t ld_in,
                                                  int32_t nt, int32_t dtype,
                                                  uint16_t *__restrict__ dst, int64_t ld_out,
                                                  int32_t col0, float *__restrict__ scale_out, int32_t dual,
                                                  int32_t *__restrict__ exp_out)
{
    __shared__ float part[256 / WAVE];
    const int64_t i = blockIdx.x;
    const float *row = src + i * ld_in;
    float m = 0.0f;
    for (int32_t n = threadIdx.x; n < nt; n += blockDim.x) m = fmaxf(m, fabsf(row[n]));
    for (int off = WAVE / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = m;
    __syncthreads();
    float mx = 0.0f;
    for (int w = 0; w < static_cast<int>(blockDim.x / WAVE); ++w) mx = fmaxf(mx, part[w]);
    float s = 1.0f;
    int32_t e = INT32_MIN;
    if (mx > 0.0f) {
        const float fr = frexpf(mx, &e);
        if (fr == 0.5f) e -= 1;          // mx is itself a power of two
        s = ldexpf(1.0f, e);
    }
    if (threadIdx.x == 0) {
        scale_out[i] = s;
        if (exp_out) exp_out[i] = e;
    }
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

// Caller-quantised 16-bit traces (binary16 or bfloat16 bits src [n_tr][ld_in]
// with power-of-two scales): one workgroup per trace writes the row in the
// dual padded layout of k_quantize (if dst is given), the scale's exponent
// (INT32_MIN when every sample is zero) and, if master is given, the
// dequantised binary32 row
// scale * q (exact) in the padded binary32 layout of k_store_f32.
__global__ __launch_bounds__(256) void k_store16(const uint16_t *__restrict__ src, int64_t ld_in, int32_t nt,
                                                 int32_t dtype, const float *__restrict__ scale,
                                                 uint16_t *__restrict__ dst, int64_t ld_out,
                                                 float *__restrict__ master, int32_t *__restrict__ exp_out)
{
    __shared__ int32_t part[256 / WAVE];
    const int64_t i = blockIdx.x;
    const uint16_t *row = src + i * ld_in;
    const float s = scale[i];
    int32_t any = 0;
    for (int32_t n = threadIdx.x; n < nt; n += blockDim.x) any |= (row[n] & 0x7fffu) != 0;
    any = __any(any) ? 1 : 0;
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = any;
    __syncthreads();
    int32_t nz = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x / WAVE); ++w) nz |= part[w];
    if (threadIdx.x == 0) {
        int32_t e = 0;
        frexpf(s, &e);
        exp_out[i] = nz ? e - 1 : INT32_MIN;   // s = 2^(e-1)
    }
    if (dst) {
        uint16_t *out = dst + i * 2 * ld_out;
        for (int64_t n = threadIdx.x; n < 2 * ld_out; n += blockDim.x) {
            const int64_t c = n < ld_out ? n : n - ld_out + 1;
            const int64_t m2 = c - PAD;
            out[n] = (m2 >= 0 && m2 < nt) ? row[m2] : static_cast<uint16_t>(0);
        }
    }
    if (master) {
        float *mrow = master + i * ld_out;
        for (int64_t n = threadIdx.x; n < ld_out; n += blockDim.x) {
            const int64_t m2 = n - PAD;
            mrow[n] = (m2 >= 0 && m2 < nt) ? s * half_to_f32(row[m2], dtype) : 0.0f;
        }
    }
}

// Relative weight scales of a bound 16-bit store, one workgroup: g = the
// largest scale exponent of a non-zero trace (0 if none); trace i gets
// 2^min(e_i - g, 0) in binary32 (rel) and, for binary16 windows, the same
// value rounded to binary16 in both halves of a dword (zero below the
// binary16 range, where a trace is more than 2^24 weaker than the strongest).
// Semblance is invariant to the common factor 2^g.
__global__ __launch_bounds__(1024) void k_relscale(const int32_t *__restrict__ e, int64_t n_tr,
                                                   float *__restrict__ rel, uint32_t *__restrict__ wsc16)
{
    __shared__ int32_t part[1024];
    int32_t g = INT32_MIN;
    for (int64_t i = threadIdx.x; i < n_tr; i += 1024) g = max(g, e[i]);
    part[threadIdx.x] = g;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] = max(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    g = part[0] == INT32_MIN ? 0 : part[0];
    for (int64_t i = threadIdx.x; i < n_tr; i += 1024) {
        const int32_t r = e[i] == INT32_MIN ? 0 : min(e[i] - g, 0);
        const float v = ldexpf(1.0f, max(r, -140));
        rel[i] = v;
        const uint32_t h = f32_to_f16_bits(v);
        wsc16[i] = h | (h << 16);
    }
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
    // the forward pass at the exact traveltimes, so that the adjoint is the
    // derivative of the interpolated semblance the binary64 definition gives
    Acc<W, float> acc;
    acc.reset();
    accumulate_range<DT, W, float, true>(sv, cand, c_lo, c_hi, 0, 1, acc);
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
    const uint32_t row_bytes = static_cast<uint32_t>(sv.ld * static_cast<int64_t>(sizeof(T)));
    // one trace's term of dS/dp, from its window
    auto grad_trace = [&](const TraceWindow<DT, W, float> &tw, float h2, float dm, float sc) {
        const TT<float> &tt = tw.tt;
        const bool use = nonzero && tt.ok && tt.tau > 0.0f;
        float u[W + 1];
        unpack_window<DT, W + 1>(tw.raw, u);
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
            g[0] += r * 2.0f * (cand.n0f + cand.As * dm) * dm * inv_dt;
            g[1] += r * cand.n0f * dm * dm * inv_dt;
            g[2] += r * cand.n0f * h2 * inv_dt;
        }
    };
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const CmpTerm<float> ct = cmp_term(cand, c, sv.dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
        int32_t i = static_cast<int32_t>(cmp_ptr[c]);
        for (; i + 1 < i1; i += 2) {
            // both windows' loads are in flight before either is used; the
            // terms are added in trace order
            const float h2a = meta[i].h2, h2b = meta[i + 1].h2;
            const TraceWindow<DT, W, float> w1 = trace_window<DT, W, float>(
                cand, ct, h2a, store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes);
            const TraceWindow<DT, W, float> w2 = trace_window<DT, W, float>(
                cand, ct, h2b, store + static_cast<size_t>(i + 1) * sv.ld, sv.copy1, row_bytes);
            grad_trace(w1, h2a, ct.dm, scale ? scale[i] : 1.0f);
            grad_trace(w2, h2b, ct.dm, scale ? scale[i + 1] : 1.0f);
        }
        if (i < i1) {
            const float h2 = meta[i].h2;
            grad_trace(trace_window<DT, W, float>(cand, ct, h2, store + static_cast<size_t>(i) * sv.ld, sv.copy1,
                                                  row_bytes),
                       h2, ct.dm, scale ? scale[i] : 1.0f);
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
                           uint16_t *dst, int64_t ld_out, int32_t col0, float *scale, bool dual, int32_t *exp_out,
                           hipStream_t s)
{
    if (n_tr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_quantize, dim3(static_cast<unsigned>(n_tr)), dim3(256), 0, s, src, ld_in, nt,
                       dtype, dst, ld_out, col0, scale, static_cast<int32_t>(dual), exp_out);
    return hipGetLastError();
}

hipError_t launch_store16(const uint16_t *src, int64_t ld_in, int64_t n_tr, int32_t nt, int32_t dtype,
                          const float *scale, uint16_t *dst, int64_t ld_out, float *master, int32_t *exp_out,
                          hipStream_t s)
{
    if (n_tr == 0) return hipSuccess;
    hipLaunchKernelGGL(k_store16, dim3(static_cast<unsigned>(n_tr)), dim3(256), 0, s, src, ld_in, nt, dtype, scale,
                       dst, ld_out, master, exp_out);
    return hipGetLastError();
}

hipError_t launch_relscale(const int32_t *e, int64_t n_tr, float *rel, uint32_t *wsc16, hipStream_t s)
{
    hipLaunchKernelGGL(k_relscale, dim3(1), dim3(1024), 0, s, e, n_tr, rel, wsc16);
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

// the search kernels of each storage type live in their own translation unit
extern template hipError_t launch_search_dt<DT_F32>(int, int, int, int, const SearchArgs &, int32_t, hipStream_t);
extern template hipError_t launch_search_dt<DT_F16>(int, int, int, int, const SearchArgs &, int32_t, hipStream_t);
extern template hipError_t launch_search_dt<DT_BF16>(int, int, int, int, const SearchArgs &, int32_t, hipStream_t);

hipError_t launch_search(int op, int dtype, int window, int kind, int dense, const SearchArgs &a,
                         int32_t n_blocks, hipStream_t s)
{
    switch (dtype) {
    case DT_F32: return launch_search_dt<DT_F32>(op, window, kind, dense, a, n_blocks, s);
    case DT_F16: return launch_search_dt<DT_F16>(op, window, kind, dense, a, n_blocks, s);
    case DT_BF16: return launch_search_dt<DT_BF16>(op, window, kind, dense, a, n_blocks, s);
    default: return hipErrorInvalidValue;
    }
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
