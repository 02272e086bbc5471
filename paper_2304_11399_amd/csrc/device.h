// Device building blocks shared by every kernel of libens (gfx950, wave64).
//
//  - Philox-4x64-10 counter-based generator (Salmon et al., SC'11).
//  - Trace store layout: each trace row holds PAD zero samples, the nt
//    samples, then zeros up to the row stride, so a window read around any
//    participating traveltime stays inside the row and reads 0 outside the
//    record without a bounds test; a trace that does not take part reads its
//    window from the leading zeros, which contributes nothing.  A 16-bit row
//    is followed by a copy of itself shifted by one sample, so that every
//    window is read as whole aligned dwords.
//  - accum_trace(): traveltime of one (candidate, trace) pair, linear
//    interpolation of the W+1 samples around it and accumulation of the
//    window sums s_k and the energy E (section "Traveltime parameter search":
//    the objective's cost is the window length times the aperture traces).
//
// The traveltime is evaluated in sample units relative to the output time
// n0 (exact integer): with tau^2 = q = n0^2 + mo, the moveout
// dtau = tau - n0 = mo / (tau + n0) is formed without cancellation, and the
// sample index n0 + floor(dtau) never goes through a rounded tau.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ens {

constexpr int PAD = 16;    // zero samples before and after each stored trace (> W)
constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Philox-4x64-10

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ---------------------------------------------------------------------------
// storage element types

enum { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

template <int DT> struct Store;
template <> struct Store<DT_F32> { using T = float; };
template <> struct Store<DT_F16> { using T = uint16_t; };
template <> struct Store<DT_BF16> { using T = uint16_t; };

__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float f16_bits_to_f32(uint32_t b)
{
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(b)));
}

typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float half_to_f32(uint32_t bits16, int DT)
{
    return DT == DT_F16 ? f16_bits_to_f32(bits16) : bf16_bits_to_f32(bits16);
}

// Raw buffer view of one padded trace row (wave-uniform, so it lives in
// scalar registers); a read past row_bytes returns zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_buffer(const void *row, uint32_t row_bytes)
{
    // word 3: 32-bit data format, no swizzle, no stride (the gfx9 raw-buffer setting)
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(row), static_cast<short>(0),
                                             static_cast<int>(row_bytes), 0x00020000);
}

// N (even for 16-bit storage) consecutive stored samples starting at byte
// `off` of row `row` (row_bytes long), as loaded (load_window_raw) and as
// binary32 (unpack_window).  16-bit rows hold a second copy shifted by one
// sample at element copy1, so a window starting at an odd element is read
// from that copy (element copy1 + off/2 - 1): always N/2 aligned dwords.  The
// loads are raw buffer loads with the row in scalar registers and a 32-bit
// lane offset.
template <int DT, int N>
struct RawWindow {
    uint32_t d[DT == DT_F32 ? N : N / 2];
};

template <int DT, int N>
__device__ __forceinline__ RawWindow<DT, N> load_window_raw(const typename Store<DT>::T *__restrict__ row,
                                                           uint32_t off, uint32_t copy1, uint32_t row_bytes)
{
    RawWindow<DT, N> r;
    const __amdgpu_buffer_rsrc_t rs = row_buffer(row, row_bytes);
    if constexpr (DT == DT_F32) {
        int k = 0;
#pragma unroll
        for (; k + 4 <= N; k += 4) {
            const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 4u * k, 0, 0);
            r.d[k] = v.x; r.d[k + 1] = v.y; r.d[k + 2] = v.z; r.d[k + 3] = v.w;
        }
        if constexpr (N % 4 >= 2) {
            const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 4u * k, 0, 0);
            r.d[k] = v.x; r.d[k + 1] = v.y;
            k += 2;
        }
        if constexpr (N % 2 == 1) r.d[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4u * k, 0, 0);
    } else {
        static_assert(N % 2 == 0, "16-bit windows hold an even number of samples");
        constexpr int ND = N / 2;
        const uint32_t start = off + (off & 2u) * (copy1 - 1u);
        int k = 0;
#pragma unroll
        for (; k + 4 <= ND; k += 4) {
            const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, start + 4u * k, 0, 0);
            r.d[k] = v.x; r.d[k + 1] = v.y; r.d[k + 2] = v.z; r.d[k + 3] = v.w;
        }
#pragma unroll
        for (; k < ND; ++k) r.d[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, start + 4u * k, 0, 0);
    }
    return r;
}

template <int DT, int N>
__device__ __forceinline__ void unpack_window(const RawWindow<DT, N> &r, float *u)
{
    if constexpr (DT == DT_F32) {
#pragma unroll
        for (int k = 0; k < N; ++k) u[k] = __uint_as_float(r.d[k]);
    } else {
#pragma unroll
        for (int m = 0; m < N / 2; ++m) {
            u[2 * m] = half_to_f32(r.d[m] & 0xffffu, DT);
            u[2 * m + 1] = half_to_f32(r.d[m] >> 16, DT);
        }
    }
}

// The per-line tables (CMP offsets, trace geometry, scales) stay unchanged
// while a kernel runs: read through the constant address space, their
// wave-uniform reads become scalar loads, which do not wait behind the
// vector memory pipe.
#define ENS_CONST_AS __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const ENS_CONST_AS T *const_view(const T *p)
{
    return (const ENS_CONST_AS T *)(p);
}

// Per-trace geometry, one 16-byte record per trace.
struct TraceMeta {
    float cx;      // CMP position c * dx
    float h2;      // h^2 (binary32)
    int32_t cmp;   // CMP index c
    float h;       // full offset
};

// Candidate constants in sample units: mo = al*dm + be*dm^2 + ga*h^2.
template <typename R>
struct Cand {
    R al, be, ga;
    R As;              // A / dt (CRS), 0 for CMP
    R n0f, n0sq;       // n0, n0^2
    R lo_lim, hi_lim;  // participation: -n0 <= dtau <= nt-1-n0
    R jx;              // output CMP position j * dx
    int32_t n0, j, ap; // output time index, output CMP, half-aperture (CMPs)
};

// Operator constants.  CMP: t^2 = t0^2 + C h^2.  CRS: t^2 = (t0 + A dm)^2 +
// B t0 dm^2 + C t0 h^2.  Divided by dt^2 with t0 = n0 dt.
template <int OP, typename R>
__device__ __forceinline__ Cand<R> make_cand(const R *p, int32_t n0, int32_t j, int32_t ap, int32_t nt,
                                             R dt, R dx)
{
    Cand<R> c;
    const R inv_dt = R(1) / dt;
    const R n0f = static_cast<R>(n0);
    if constexpr (OP == 1) {
        c.al = R(0);
        c.be = R(0);
        c.ga = p[0] * inv_dt * inv_dt;
        c.As = R(0);
    } else {
        const R As = p[0] * inv_dt;            // A / dt  (samples per metre)
        c.al = R(2) * n0f * As;
        c.be = As * As + p[1] * n0f * inv_dt;  // (A/dt)^2 + B t0 / dt^2
        c.ga = p[2] * n0f * inv_dt;            // C t0 / dt^2
        c.As = As;
    }
    c.n0f = n0f;
    c.n0sq = n0f * n0f;
    c.lo_lim = -n0f;
    c.hi_lim = static_cast<R>(nt - 1 - n0);
    c.jx = static_cast<R>(j) * dx;
    c.n0 = n0;
    c.j = j;
    c.ap = ap;
    return c;
}

template <int W, typename R>
struct Acc {
    R s[W];
    R E;
    int32_t M;
    __device__ __forceinline__ void reset()
    {
#pragma unroll
        for (int k = 0; k < W; ++k) s[k] = R(0);
        E = R(0);
        M = 0;
    }
};

// Fused multiply-add in the operands' own precision.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float floor_r(float x) { return __builtin_floorf(x); }
__device__ __forceinline__ double floor_r(double x) { return __builtin_floor(x); }
// Clamp into [lo, hi]; a NaN gives a bound, which differs from the NaN.
__device__ __forceinline__ float clamp_to(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }
__device__ __forceinline__ double clamp_to(double x, double lo, double hi)
{
    return __builtin_fmin(__builtin_fmax(x, lo), hi);
}

__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

// Per-CMP part of the moveout for one candidate: al dm + be dm^2 with
// dm = (c - j) dx, and whether the CMP lies inside the candidate's aperture.
template <typename R>
struct CmpTerm {
    R part;
    R Q;          // n0^2 + part: q = Q + ga h^2
    R dm;
    bool in_ap;
};

template <typename R>
__device__ __forceinline__ CmpTerm<R> cmp_term(const Cand<R> &cand, int32_t c, R dx)
{
    CmpTerm<R> t;
    const int32_t dc = c - cand.j;
    t.dm = static_cast<R>(dc) * dx;
    t.part = fmadd(cand.be, t.dm * t.dm, cand.al * t.dm);
    t.Q = cand.n0sq + t.part;
    t.in_ap = dc <= cand.ap && -dc <= cand.ap;
    return t;
}

// Traveltime of (candidate, trace) in sample units.  q = n0^2 + mo < 0 (no
// real traveltime) fails the range test, as does any trace outside the
// candidate's aperture.  off: byte offset of the window's first sample in the
// padded row of ESZ-byte elements, or 0 (a run of zero padding) for a trace
// that does not take part.
template <typename R>
struct TT {
    bool ok;
    uint32_t off;
    R f;
    R tau;        // sqrt(q) in samples
};

template <int W, int ESZ, typename R>
__device__ __forceinline__ TT<R> traveltime(const Cand<R> &c, const CmpTerm<R> &ct, R h2)
{
    static_assert(ESZ == 2 || ESZ == 4, "2- or 4-byte samples");
    TT<R> r;
    const R mo = fmadd(c.ga, h2, ct.part);
    const R q = c.n0sq + mo;
    // q < 0: the square root is NaN, the guarded denominator 1e-30 and dtau
    // a large negative number (mo < -n0^2 <= 0), below every range
    const R tau = fast_sqrt(q);
    const R s = tau + c.n0f;
    const R den = s > R(1e-30) ? s : R(1e-30);
    const R dtau = mo * fast_rcp(den);
    // participation -n0 <= dtau <= nt-1-n0: the clamped value equals dtau
    // exactly when dtau lies in the range; the clamped value keeps the
    // fraction and the window column finite for every trace
    const R dc = clamp_to(dtau, c.lo_lim, c.hi_lim);
    r.ok = ct.in_ap && dc == dtau;
    const R fl = floor_r(dc);
    r.f = dc - fl;
    uint32_t off;
    if constexpr (sizeof(R) == 4) {
        // column n0 + fl + PAD - W/2 lies in [0, nt + PAD) with nt <= 2^20:
        // adding it to 1.5 * 2^23 is exact and gives the bit pattern
        // 0x4B400000 + column, so the column needs no float-to-integer
        // conversion (the constant part is per candidate)
        const float K = c.n0f + (12582912.0f + static_cast<float>(PAD - W / 2));
        const uint32_t bits = __float_as_uint(fl + K);
        off = bits * ESZ - 0x4B400000u * ESZ;
    } else {
        off = static_cast<uint32_t>(c.n0 + static_cast<int32_t>(fl) + (PAD - W / 2)) * ESZ;
    }
    r.off = r.ok ? off : 0u;
    r.tau = tau;
    return r;
}

// One trace's window in two halves, so that a caller can issue the loads of
// two traces before it uses either: the traveltime and the window load, then
// the interpolation and the sums.  row: the padded trace row, row_bytes long.
template <int DT, int W, typename R>
struct TraceWindow {
    TT<R> tt;
    RawWindow<DT, W + 1> raw;
};

template <int DT, int W, typename R>
__device__ __forceinline__ TraceWindow<DT, W, R> trace_window(const Cand<R> &c, const CmpTerm<R> &ct, R h2,
                                                              const typename Store<DT>::T *__restrict__ row,
                                                              uint32_t copy1, uint32_t row_bytes)
{
    TraceWindow<DT, W, R> r;
    r.tt = traveltime<W, sizeof(typename Store<DT>::T)>(c, ct, h2);
    r.raw = load_window_raw<DT, W + 1>(row, r.tt.off, copy1, row_bytes);
    return r;
}

template <int DT, int W, bool SCALED, typename R>
__device__ __forceinline__ void trace_accumulate(Acc<W, R> &acc, const TraceWindow<DT, W, R> &tw, float scale)
{
    const TT<R> &tt = tw.tt;
    R wb = tt.f;
    R wa = R(1) - tt.f;
    if constexpr (SCALED) {
        wa *= static_cast<R>(scale);
        wb *= static_cast<R>(scale);
    }
    acc.M += tt.ok ? 1 : 0;
    float u[W + 1];
    unpack_window<DT, W + 1>(tw.raw, u);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        // binary32 samples in binary32: u_k + f (u_k+1 - u_k), a difference
        // and one fused step, with no separate 1 - f; binary16 samples: two
        // fused steps, so that they feed the mixed-precision FMA without a
        // separate conversion (measured faster than converting first);
        // otherwise a product and one fused step
        R a;
        if constexpr (DT == DT_F32 && !SCALED && sizeof(R) == 4)
            a = fmadd(tt.f, u[k + 1] - u[k], u[k]);
        else if constexpr (DT == DT_F16)
            a = fmadd(wb, static_cast<R>(u[k + 1]), fmadd(wa, static_cast<R>(u[k]), R(0)));
        else
            a = fmadd(wb, static_cast<R>(u[k + 1]), wa * static_cast<R>(u[k]));
        acc.s[k] += a;
        acc.E = fmadd(a, a, acc.E);
    }
}

template <int DT, int W, bool SCALED, typename R>
__device__ __forceinline__ void accum_trace(Acc<W, R> &acc, const Cand<R> &c, const CmpTerm<R> &ct,
                                            R h2, const typename Store<DT>::T *__restrict__ row,
                                            uint32_t copy1, uint32_t row_bytes, float scale)
{
    trace_accumulate<DT, W, SCALED, R>(acc, trace_window<DT, W, R>(c, ct, h2, row, copy1, row_bytes), scale);
}

// A VALU instruction may read the result of v_dot2_f32_f16 only three wait
// states after it.  The compiler counts them for its own instructions but not
// for inline assembly, so every dot result passes through one s_nop 2 (three
// wait states) before anything reads it.  The statement is not volatile: its
// operands order it after the dots and before every reader, and a volatile
// statement would also stop the scheduler from moving the next trace's load
// above it.
template <int W>
__device__ __forceinline__ void dot_results_ready(float *a)
{
    static_assert(W % 2 == 1 && W >= 3 && W <= 15, "odd window, 3..15");
    if constexpr (W == 3) {
        asm("s_nop 2" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]));
    } else if constexpr (W == 5) {
        asm("s_nop 2" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]));
    } else if constexpr (W == 7) {
        asm("s_nop 2" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]),
                     "+v"(a[6]));
    } else {
        // longer windows: the first seven, then the rest
        asm("s_nop 2" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]),
                     "+v"(a[6]));
        dot_results_ready<W - 6>(a + 6);
    }
}

// Binary16 windows through packed dot products.  The traveltime in samples
// tau = sqrt(q) is rounded to the grid of spacing 2^-11 (B = 4096; 2^-10 and
// 2^-9 for records of up to 8176 and 16368 samples, the longest that binary16
// windows take) by one binary32 addition: y = tau + B + PAD - W/2 lies in
// [B, 2B), where binary32 values are spaced by the grid.  floor(y) - B is the
// window's first column and wb = y - floor(y), wa = 1 - wb are exact multiples
// of the grid, hence exact in binary16, as are their products with the
// trace's power-of-two weight scale.  Each interpolated sample is then one
// v_dot2_f32_f16 of the stored pair (u_k, u_k+1) with (wa, wb): binary16
// products are exact in binary32, so a_k carries no rounding beyond the
// binary32 sum.  Pairs (u_k, u_k+1) with k odd straddle two dwords and are
// taken with alignbit.  A trace that does not take part (q < 0, tau > nt - 1,
// outside the aperture) gets zero weights, which also clears whatever the
// window load returned.
// One trace's binary16 window in two halves, so that a caller can issue the
// loads of two traces before it uses either: the traveltime, the weights and
// the window load, then the dot products and the sums.
template <int W>
struct F16Window {
    uint32_t d[(W + 1) / 2];
    uint32_t wbits;
};

template <int W>
__device__ __forceinline__ F16Window<W> f16_window(Acc<W, float> &acc, const CmpTerm<float> &ct, float ga, float h2,
                                                   const uint16_t *__restrict__ row, uint32_t copy1,
                                                   uint32_t row_bytes, uint32_t wsc, const float kq, uint32_t bbits,
                                                   uint32_t shift, float tau_max)
{
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    constexpr int ND = (W + 1) / 2;
    F16Window<W> r;
    const float q = fmadd(ga, h2, ct.Q);
    const float tau = fast_sqrt(q);
    // tau_max: the record's last sample, or -1 where the CMP lies outside the
    // candidate's aperture; false for a NaN (q < 0)
    const bool ok = tau <= tau_max;
    const float y = tau + kq;
    const float fl = floor_r(y);
    const float wb = y - fl;
    const float wa = 1.0f - wb;
    const uint32_t off = (__float_as_uint(fl) - bbits) >> shift;   // 2 * column, in bytes
    const uint32_t start = off + __umul24(off & 2u, copy1 - 1u);
    half2_t w = __builtin_bit_cast(half2_t, __builtin_amdgcn_cvt_pkrtz(wa, wb));
    w = w * __builtin_bit_cast(half2_t, wsc);
    r.wbits = ok ? __builtin_bit_cast(uint32_t, w) : 0u;
    acc.M += ok ? 1 : 0;
    const __amdgpu_buffer_rsrc_t rs = row_buffer(row, row_bytes);
    int m = 0;
#pragma unroll
    for (; m + 4 <= ND; m += 4) {
        const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, start + 4u * m, 0, 0);
        r.d[m] = v.x; r.d[m + 1] = v.y; r.d[m + 2] = v.z; r.d[m + 3] = v.w;
    }
    if constexpr (ND % 4 >= 2) {
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, start + 4u * m, 0, 0);
        r.d[m] = v.x; r.d[m + 1] = v.y;
        m += 2;
    }
    if constexpr (ND % 2 == 1) r.d[m] = __builtin_amdgcn_raw_buffer_load_b32(rs, start + 4u * m, 0, 0);
    return r;
}

template <int W>
__device__ __forceinline__ void f16_accumulate(Acc<W, float> &acc, const F16Window<W> &win)
{
    float a[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t pr =
            (k & 1) ? __builtin_amdgcn_alignbit(win.d[k / 2 + 1], win.d[k / 2], 16) : win.d[k / 2];
        // the three-operand form with an inline zero (the two-operand form the
        // compiler picks for a zero accumulator costs a register clear each)
        asm("v_dot2_f32_f16 %0, %1, %2, 0" : "=v"(a[k]) : "v"(pr), "v"(win.wbits));
    }
    dot_results_ready<W>(a);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        acc.s[k] += a[k];
        acc.E = fmadd(a[k], a[k], acc.E);
    }
}

template <int W>
__device__ __forceinline__ void accum_trace_f16(Acc<W, float> &acc, const CmpTerm<float> &ct, float ga, float h2,
                                                const uint16_t *__restrict__ row, uint32_t copy1, uint32_t row_bytes,
                                                uint32_t wsc, const float kq, uint32_t bbits, uint32_t shift,
                                                float tau_max)
{
    f16_accumulate<W>(acc, f16_window<W>(acc, ct, ga, h2, row, copy1, row_bytes, wsc, kq, bbits, shift, tau_max));
}

template <int W, typename R>
__device__ __forceinline__ R finish_semblance(const Acc<W, R> &acc)
{
    R N = R(0);
#pragma unroll
    for (int k = 0; k < W; ++k) N = fmadd(acc.s[k], acc.s[k], N);
    if (acc.M > 0 && acc.E > R(0)) return N / (static_cast<R>(acc.M) * acc.E);
    return R(0);
}

// ---------------------------------------------------------------------------
// evolution step (binary32 arithmetic written out operation by operation;
// the library is built without floating-point contraction)

struct TrialDraw {
    uint32_t r1, r2, jr;
    bool take[3];
};

// Indices and crossover decisions of one slot from its generator block.  r2
// ranges over a pool of np members plus any archive entries (indices from
// np on), excluding the slot itself and r1.
__device__ __forceinline__ TrialDraw trial_draw(const uint64_t w[4], int32_t i, int32_t np, int32_t P,
                                                uint64_t cr_thr, int32_t pool)
{
    TrialDraw d;
    uint32_t r1 = static_cast<uint32_t>(((w[0] >> 32) * static_cast<uint64_t>(np - 1)) >> 32);
    if (r1 >= static_cast<uint32_t>(i)) r1 += 1;
    uint32_t r2 = static_cast<uint32_t>(((w[0] & 0xffffffffULL) * static_cast<uint64_t>(pool - 2)) >> 32);
    const uint32_t ui = static_cast<uint32_t>(i);
    const uint32_t ex_lo = ui < r1 ? ui : r1, ex_hi = ui < r1 ? r1 : ui;
    if (r2 >= ex_lo) r2 += 1;
    if (r2 >= ex_hi) r2 += 1;
    d.r1 = r1;
    d.r2 = r2;
    d.jr = static_cast<uint32_t>(((w[1] >> 32) * static_cast<uint64_t>(P)) >> 32);
    const uint64_t cr[3] = {w[1] & 0xffffffffULL, w[2] >> 32, w[2] & 0xffffffffULL};
#pragma unroll
    for (int k = 0; k < 3; ++k) d.take[k] = cr[k] < cr_thr || static_cast<uint32_t>(k) == d.jr;
    return d;
}

// Mutant coordinate, repaired into [lo, hi] by the midpoint toward the parent.
__device__ __forceinline__ float mutant(float xi, float xb, float xr1, float xr2, float F, float lo,
                                        float hi)
{
    const float t1 = xb - xi;
    const float t2 = xr1 - xr2;
    const float m1 = F * t1;
    const float m2 = F * t2;
    float v = xi + m1;
    v = v + m2;
    if (v < lo)
        v = (lo + xi) * 0.5f;
    else if (v > hi)
        v = (hi + xi) * 0.5f;
    return v;
}

// JADE control parameters of one slot from its adaptation block (the same
// definition as the oracle's): CR ~ N(mu_CR, 0.1) clipped to [0, 1] by
// Box-Muller, F ~ Cauchy(mu_F, 0.1) by the inverse CDF, 1 where above 1,
// redrawn where not positive (three draws, then mu_F); both on the grid
// k / 2^24.  a_idx: archive position a replaced parent overwrites when the
// archive is full.  Binary64 throughout.  The logarithm, sine and cosine are
// series on reduced arguments written out operation by operation (ln u =
// e ln 2 + 2 atanh((m-1)/(m+1)) with m in [sqrt(1/2), sqrt(2)) and atanh to
// the s^23 term; sin and cos on [0, pi/2] by Taylor series to a^25, a^24):
// no library routine, so the bits do not depend on a math library, and few
// registers.
constexpr double JADE_GRID = 16777216.0;
constexpr double JADE_PI = 3.14159265358979323846;

__device__ __forceinline__ double jade_ln(double u)
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
#pragma unroll
    for (int k = 21; k >= 1; k -= 2) p = p * s2 + 1.0 / static_cast<double>(k);
    return static_cast<double>(e) * 0.693147180559945309417 + 2.0 * s * p;
}

__device__ __forceinline__ void jade_sincos(double a, double &sn, double &cs)
{
    const double a2 = a * a;
    double ps = 1.0, pc = 1.0;
#pragma unroll
    for (int k = 24; k >= 2; k -= 2) {
        ps = 1.0 - ps * a2 / static_cast<double>(k * (k + 1));
        pc = 1.0 - pc * a2 / static_cast<double>((k - 1) * k);
    }
    sn = a * ps;
    cs = pc;
}

__device__ __forceinline__ void jade_draws(const uint64_t w[4], double mu_cr, double mu_f, int32_t np,
                                           int32_t &k_cr, int32_t &k_f, int32_t &a_idx)
{
    const double u1 = (static_cast<double>(w[0] >> 11) + 1.0) * 0x1p-53;
    const double u2 = static_cast<double>(w[1] >> 11) * 0x1p-53;
    // cos(2 pi u2) from the quarter turn and the angle within it
    const double v = 4.0 * u2;
    const double q = floor(v);
    double sn, cs;
    jade_sincos((v - q) * (JADE_PI / 2.0), sn, cs);
    const int iq = static_cast<int>(q);
    const double c2 = iq == 0 ? cs : (iq == 1 ? -sn : (iq == 2 ? -cs : sn));
    const double z = sqrt(-2.0 * jade_ln(u1)) * c2;
    double cr = mu_cr + 0.1 * z;
    cr = cr < 0.0 ? 0.0 : cr;
    cr = cr > 1.0 ? 1.0 : cr;
    k_cr = static_cast<int32_t>(rint(cr * JADE_GRID));
    const uint64_t h[3] = {w[2] >> 32, w[2] & 0xffffffffULL, w[3] >> 32};
    int32_t kf = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (kf == 0) {
            const double u = (static_cast<double>(h[a]) + 0.5) * 0x1p-32;
            const double x = u - 0.5;  // tan(pi x) = sign(x) sin(pi |x|) / cos(pi |x|)
            double sx, cx;
            jade_sincos((x < 0.0 ? -x : x) * JADE_PI, sx, cx);
            const double tx = sx / cx;
            double f = mu_f + 0.1 * (x < 0.0 ? -tx : tx);
            f = f > 1.0 ? 1.0 : f;
            if (f > 0.0) kf = static_cast<int32_t>(rint(f * JADE_GRID));
        }
    }
    if (kf == 0) {
        kf = static_cast<int32_t>(rint(mu_f * JADE_GRID));
        kf = kf < 1 ? 1 : kf;
    }
    k_f = kf;
    a_idx = static_cast<int32_t>(((w[3] & 0xffffffffULL) * static_cast<uint64_t>(np)) >> 32);
}

__device__ __forceinline__ float init_coord(uint64_t w, float lo, float hi)
{
    const float u = static_cast<float>(w >> 40) * 0x1p-24f;
    const float range = hi - lo;
    const float step = u * range;
    return lo + step;
}

// XCD-aware block order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; give each XCD a contiguous run of work items so that the
// traces those items gather stay in that XCD's L2.
__device__ __forceinline__ int32_t xcd_remap(int32_t bid, int32_t nblocks)
{
    constexpr int NX = 8;
    const int32_t per = nblocks / NX, rem = nblocks % NX;
    const int32_t x = bid % NX, local = bid / NX;
    return x * per + (x < rem ? x : rem) + local;
}

}  // namespace ens
