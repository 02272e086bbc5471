// Semblance accumulation shared by the kernels of libens: wave helpers, the
// trace loop over a candidate's aperture, and the compile-time dispatch
// macros of the launch wrappers.
#pragma once

#include "device.h"
#include "launch.h"

namespace ens {

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
// EXACT: binary16 windows through the binary32 interpolation of the
// converted samples at the exact traveltime (the adjoint's forward pass),
// instead of the packed dot products on the 2^-11-sample grid.
template <int DT, int W, bool SCALED, typename R, bool EXACT = false>
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
    if constexpr (DT == DT_F16 && sizeof(R) == 4 && !EXACT) {
        const ENS_CONST_AS uint32_t *wsc = const_view(sv.wsc16);
        // kq and bbits in vector registers: a scalar operand halves the issue
        // rate of the addition and subtraction that use them
        float kq;
        uint32_t bbits;
        asm("v_mov_b32 %0, %1" : "=v"(kq) : "s"(sv.h16_kq));
        asm("v_mov_b32 %0, %1" : "=v"(bbits) : "s"(sv.h16_bbits));
        const float tau_max = sv.tau_max;
        const uint32_t shift = sv.h16_shift;
        for (int32_t c = c_lo; c <= c_hi; ++c) {
            const CmpTerm<R> ct = cmp_term(cand, c, dx);
            // the aperture test folded into the record test: tau <= -1 never holds
            const float tmax = ct.in_ap ? tau_max : -1.0f;
            const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
            int32_t i = static_cast<int32_t>(cmp_ptr[c]) + first;
            for (; i + step < i1; i += 2 * step) {
                // both windows' loads are in flight before either is used
                const int32_t i2 = i + step;
                const F16Window<W> w1 = f16_window<W>(acc, ct, cand.ga, meta[i].h2,
                                                      store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes,
                                                      wsc[i], kq, bbits, shift, tmax);
                const F16Window<W> w2 = f16_window<W>(acc, ct, cand.ga, meta[i2].h2,
                                                      store + static_cast<size_t>(i2) * sv.ld, sv.copy1, row_bytes,
                                                      wsc[i2], kq, bbits, shift, tmax);
                f16_accumulate<W>(acc, w1);
                f16_accumulate<W>(acc, w2);
            }
            if (i < i1)
                accum_trace_f16<W>(acc, ct, cand.ga, meta[i].h2, store + static_cast<size_t>(i) * sv.ld, sv.copy1,
                                   row_bytes, wsc[i], kq, bbits, shift, tmax);
        }
        return;
    }
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const CmpTerm<R> ct = cmp_term(cand, c, dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
        int32_t i = static_cast<int32_t>(cmp_ptr[c]) + first;
        for (; i + step < i1; i += 2 * step) {
            // both windows' loads are in flight before either is used
            const int32_t i2 = i + step;
            const TraceWindow<DT, W, R> w1 = trace_window<DT, W, R>(
                cand, ct, h2_of<R>(meta, i), store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes);
            const TraceWindow<DT, W, R> w2 = trace_window<DT, W, R>(
                cand, ct, h2_of<R>(meta, i2), store + static_cast<size_t>(i2) * sv.ld, sv.copy1, row_bytes);
            trace_accumulate<DT, W, SCALED, R>(acc, w1, SCALED ? scale[i] : 1.0f);
            trace_accumulate<DT, W, SCALED, R>(acc, w2, SCALED ? scale[i2] : 1.0f);
        }
        if (i < i1)
            accum_trace<DT, W, SCALED>(acc, cand, ct, h2_of<R>(meta, i),
                                       store + static_cast<size_t>(i) * sv.ld, sv.copy1, row_bytes,
                                       SCALED ? scale[i] : 1.0f);
    }
}

// Binary32 windows through LDS: tab[i - i0] = {first column, columns} of the
// range every window of trace i may read for the workgroup's candidates
// (columns < 0: read directly); stage: this wave's 2 x (TILE_STAGE_MAX + 8)
// floats; zero8: 8 zero floats.  The staged samples and the arithmetic are
// those of accum_trace, so the sums are bit for bit those of the direct path.
template <int W>
__device__ __forceinline__ void accumulate_cmps_tiles(const StoreView &sv, const Cand<float> &cand, int32_t c_lo,
                                                      int32_t c_hi, int32_t first, int32_t step,
                                                      Acc<W, float> &acc, const int2 *tab, int32_t i0,
                                                      float *stage, const float *zero8, int32_t lane)
{
    const float *store = static_cast<const float *>(sv.store);
    const ENS_CONST_AS int64_t *cmp_ptr = const_view(sv.cmp_ptr);
    const ENS_CONST_AS TraceMeta *meta = const_view(sv.meta);
    const float dx = sv.dx;
    const uint32_t row_bytes = static_cast<uint32_t>(sv.ld * static_cast<int64_t>(sizeof(float)));
    auto one = [&](const CmpTerm<float> &ct, int32_t i, float *buf) {
        const float *row = store + static_cast<size_t>(i) * sv.ld;
        const int2 te = tab[i - i0];
        const int32_t b = __builtin_amdgcn_readfirstlane(te.x), len = __builtin_amdgcn_readfirstlane(te.y);
        if (len < 0) {
            accum_trace<DT_F32, W, false>(acc, cand, ct, meta[i].h2, row, 0u, row_bytes, 1.0f);
            return;
        }
        const __amdgpu_buffer_rsrc_t rs = row_buffer(row, row_bytes);
#pragma unroll
        for (int r = 0; r < TILE_STAGE_MAX; r += WAVE)
            if (r < len) buf[r + lane] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                                             rs, static_cast<uint32_t>(b + r + lane) * 4u, 0, 0));
        __builtin_amdgcn_wave_barrier();
        const TT<float> tt = traveltime<W, 4>(cand, ct, meta[i].h2);
        acc.M += tt.ok ? 1 : 0;
        // tt.off is 4 * column for a participating trace
        const float *src = tt.ok ? buf + (static_cast<int32_t>(tt.off >> 2) - b) : zero8;
        float u[W + 1];
#pragma unroll
        for (int k = 0; k <= W; ++k) u[k] = src[k];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const float a = fmadd(tt.f, u[k + 1] - u[k], u[k]);
            acc.s[k] += a;
            acc.E = fmadd(a, a, acc.E);
        }
        __builtin_amdgcn_wave_barrier();
    };
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const CmpTerm<float> ct = cmp_term(cand, c, dx);
        const int32_t i1 = static_cast<int32_t>(cmp_ptr[c + 1]);
        int32_t i = static_cast<int32_t>(cmp_ptr[c]) + first;
        for (; i + step < i1; i += 2 * step) {
            one(ct, i, stage);
            one(ct, i + step, stage + TILE_STAGE_MAX + 8);
        }
        if (i < i1) one(ct, i, stage);
    }
}

template <int DT, int W, typename R, bool EXACT = false>
__device__ __forceinline__ void accumulate_range(const StoreView &sv, const Cand<R> &cand, int32_t c_lo,
                                                 int32_t c_hi, int32_t first, int32_t step,
                                                 Acc<W, R> &acc)
{
    if constexpr (DT == DT_F16)
        accumulate_cmps<DT, W, true, R, EXACT>(sv, cand, c_lo, c_hi, first, step, acc);
    else if (sv.scale)
        accumulate_cmps<DT, W, true, R>(sv, cand, c_lo, c_hi, first, step, acc);
    else
        accumulate_cmps<DT, W, false, R>(sv, cand, c_lo, c_hi, first, step, acc);
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

}  // namespace ens
