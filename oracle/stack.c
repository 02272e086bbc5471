/*
 * Zero-offset stack along each sample's operator, and the RMS of a panel, in
 * binary64.  Test infrastructure (see oracle.h).
 *
 * Section "Traveltime parameter search": the operators exist to stack a
 * sample, i.e. to combine the amplitudes that the operator's curve picks in
 * the traces of the aperture; section "Qualitative analysis" shows the
 * stacked panels next to the coherence panels, and section "Quantitative
 * analysis" compares methods by the RMS of the coherence panels.  Neither
 * formula is printed.  Readings used here:
 *   stack(j, n0; p) = (1/M) sum_i ((1-f_i) u_i[n_i] + f_i u_i[n_i+1])
 * over the M traces that take part in the semblance of (j, n0; p) (same
 * aperture, same participation rule, tau_i = n_i + f_i), 0 when M = 0: the
 * amplitude of the window's centre sample, averaged over the fold;
 *   rms(x) = sqrt(sum_k x_k^2 / n), 0 for n = 0.
 */
#include <math.h>

#include "oracle.h"

static double sample_at(const or_line *L, int64_t i, int64_t m)
{
    if (m < 0 || m >= L->nt)
        return 0.0;
    return L->u[i * (int64_t)L->nt + m];
}

double or_stack(const or_line *L, int32_t j, int32_t n0, const double *p, int32_t *M_out)
{
    const int32_t a = or_aperture(L, n0);
    const int32_t c_lo = j - a < 0 ? 0 : j - a;
    const int32_t c_hi = j + a > L->n_cmp - 1 ? L->n_cmp - 1 : j + a;
    const double t0 = (double)n0 * L->dt;
    double sum = 0.0;
    int32_t M = 0;
    for (int32_t c = c_lo; c <= c_hi; ++c) {
        const double dm = (double)(c - j) * L->dx;
        for (int64_t i = L->cmp_ptr[c]; i < L->cmp_ptr[c + 1]; ++i) {
            const double h = L->offset[i];
            double q;
            if (L->op == 1) {
                q = t0 * t0 + p[0] * h * h;
            } else {
                const double lin = t0 + p[0] * dm;
                q = lin * lin + p[1] * t0 * dm * dm + p[2] * t0 * h * h;
            }
            if (q < 0.0)
                continue;
            const double tau = sqrt(q) / L->dt;
            if (tau > (double)(L->nt - 1))
                continue;
            const int64_t n = (int64_t)floor(tau);
            const double f = tau - (double)n;
            sum += (1.0 - f) * sample_at(L, i, n) + f * sample_at(L, i, n + 1);
            M += 1;
        }
    }
    if (M_out)
        *M_out = M;
    return M > 0 ? sum / (double)M : 0.0;
}

void or_stack_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                    const double *params, double *out, int32_t *M)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n; ++c) {
        int32_t m = 0;
        out[c] = or_stack(L, cmp[c], t[c], params + c * P, &m);
        if (M)
            M[c] = m;
    }
}

double or_rms(const double *x, int64_t n)
{
    if (n <= 0)
        return 0.0;
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k)
        s += x[k] * x[k];
    return sqrt(s / (double)n);
}
