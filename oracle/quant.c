/*
 * Per-trace scaled binary16 / bfloat16 trace storage, written out bit by bit
 * from the IEEE 754 binary16 format and the bfloat16 format (binary32 with
 * the low 16 mantissa bits dropped).  Test infrastructure (see oracle.h).
 *
 * scale_i = the smallest power of two at or above max_n |u_i[n]| (1 when the
 * trace is all zero); q_i[n] = round-to-nearest-even(u_i[n] / scale_i), the
 * quotient exact in binary32.  A power-of-two scale leaves the relative
 * precision of the floating-point formats unchanged and makes s_i q_i[n]
 * exact, so the scale can be applied to interpolation weights without
 * rounding.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

static uint32_t f32_bits(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    return x;
}

static uint16_t f32_to_f16_rne(float f)
{
    uint32_t x = f32_bits(f);
    uint16_t sign = (uint16_t)((x >> 16) & 0x8000u);
    uint32_t ax = x & 0x7fffffffu;
    if (ax >= 0x7f800000u) /* inf or nan */
        return sign | (ax > 0x7f800000u ? 0x7e00u : 0x7c00u);
    if (ax >= 0x477ff000u) /* rounds past the largest finite binary16 */
        return sign | 0x7c00u;
    if (ax < 0x38800000u) {
        /* binary16 subnormal: value = m 2^-24 with m = round-half-even(|f| 2^24) */
        double v = fabs((double)f) * 16777216.0;
        double m = floor(v);
        double r = v - m;
        if (r > 0.5 || (r == 0.5 && fmod(m, 2.0) != 0.0))
            m += 1.0;
        return sign | (uint16_t)m;
    }
    uint32_t e = (ax >> 23) - 127u + 15u;
    uint32_t mant = ax & 0x7fffffu;
    uint32_t h = (e << 10) | (mant >> 13);
    uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u)))
        h += 1u; /* a carry into the exponent is the correct rounding */
    return sign | (uint16_t)h;
}

static uint16_t f32_to_bf16_rne(float f)
{
    uint32_t x = f32_bits(f);
    if ((x & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((x >> 16) | 0x40u);
    uint32_t lsb = (x >> 16) & 1u;
    return (uint16_t)((x + 0x7fffu + lsb) >> 16);
}

double or_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(m | 0x400), e - 25);
    return sign ? -v : v;
}

double or_bf16_to_double(uint16_t h)
{
    uint32_t x = (uint32_t)h << 16;
    float f;
    memcpy(&f, &x, 4);
    return (double)f;
}

void or_quantize(const float *u, int64_t n_tr, int32_t nt, int32_t dtype, uint16_t *q,
                 float *scale)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_tr; ++i) {
        const float *row = u + i * nt;
        float s = 0.0f;
        for (int32_t n = 0; n < nt; ++n)
            if (fabsf(row[n]) > s)
                s = fabsf(row[n]);
        if (s == 0.0f) {
            s = 1.0f;
        } else {
            int e = 0;
            const float fr = frexpf(s, &e); /* s = fr 2^e, fr in [1/2, 1) */
            s = fr == 0.5f ? s : ldexpf(1.0f, e);
        }
        scale[i] = s;
        for (int32_t n = 0; n < nt; ++n) {
            float x = row[n] / s;
            q[i * nt + n] = dtype == 1 ? f32_to_f16_rne(x) : f32_to_bf16_rne(x);
        }
    }
}
