/*
 * Traveltime operators, linearly interpolated gather, windowed semblance and
 * its gradient, in binary64.  Test infrastructure (see oracle.h).
 *
 * The objective is the semblance coherence of the paper's section
 * "Traveltime parameter search" (eqs. f, S, Sf: a map onto [0,1] of the
 * parameters, the data and the configuration, whose cost is linear in the
 * window length times the traces in the aperture, eq. order).  The paper
 * cites Neidell & Taner for it without printing it; the standard definition
 * is used:  for the M participating traces i of the aperture and the window
 * offsets k = -w..w around each trace's traveltime,
 *     a_ik = (1-f_i) u_i[n_i+k] + f_i u_i[n_i+k+1],   tau_i = n_i + f_i,
 *     s_k = sum_i a_ik,  E = sum_k sum_i a_ik^2,  N = sum_k s_k^2,
 *     S = N / (M E)   (S = 0 when M = 0 or E = 0),
 * which lies in [0,1] by Cauchy-Schwarz.  Samples outside the record read 0.
 *
 * Operators (section "Traveltime parameter search"; CMP needs one velocity
 * parameter, CRS uses midpoint displacements from neighbouring traces):
 *     CMP: t^2 = t0^2 + C h^2
 *     CRS: t^2 = (t0 + A dm)^2 + B t0 dm^2 + C t0 h^2
 * with h the full offset, dm the midpoint displacement of the trace's CMP
 * from the output CMP and t0 = n0 dt.  A trace takes part iff t^2 >= 0 and
 * 0 <= t/dt <= nt-1.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

int32_t or_aperture(const or_line *L, int32_t n0)
{
    if (L->nt <= 1)
        return L->ap_lo;
    double a = L->ap_lo + (double)(L->ap_hi - L->ap_lo) * (double)n0 / (double)(L->nt - 1);
    return (int32_t)floor(a + 0.5);
}

static double sample_at(const or_line *L, int64_t i, int64_t m)
{
    if (m < 0 || m >= L->nt)
        return 0.0;
    return L->u[i * (int64_t)L->nt + m];
}

/* Squared traveltime q and its partial derivatives dq/dp. */
static double traveltime_sq(const or_line *L, const double *p, double t0, double dm, double h,
                            double *dq)
{
    if (L->op == 1) {
        if (dq)
            dq[0] = h * h;
        return t0 * t0 + p[0] * h * h;
    }
    double A = p[0], B = p[1], C = p[2];
    double lin = t0 + A * dm;
    if (dq) {
        dq[0] = 2.0 * lin * dm;
        dq[1] = t0 * dm * dm;
        dq[2] = t0 * h * h;
    }
    return lin * lin + B * t0 * dm * dm + C * t0 * h * h;
}

/* Shared walk over the aperture: fills the window sums, and optionally the
 * gradient in a second pass once S is known. */
static double semblance_impl(const or_line *L, int32_t j, int32_t n0, const double *p,
                             int32_t *M_out, double *margin_out, double *grad, double *tau_l1)
{
    const int w = L->half_w, W = 2 * w + 1;
    const int P = L->op;
    const int32_t a = or_aperture(L, n0);
    const int32_t c_lo = j - a < 0 ? 0 : j - a;
    const int32_t c_hi = j + a > L->n_cmp - 1 ? L->n_cmp - 1 : j + a;
    const double t0 = (double)n0 * L->dt;
    double *s = calloc((size_t)W, sizeof(double));
    double E = 0.0, margin = INFINITY;
    int32_t M = 0;

    for (int32_t c = c_lo; c <= c_hi; ++c) {
        double dm = (double)(c - j) * L->dx;
        for (int64_t i = L->cmp_ptr[c]; i < L->cmp_ptr[c + 1]; ++i) {
            double q = traveltime_sq(L, p, t0, dm, L->offset[i], NULL);
            double tau_signed = (q >= 0.0 ? sqrt(q) : -sqrt(-q)) / L->dt;
            if (fabs(tau_signed) < margin)
                margin = fabs(tau_signed);
            if (q < 0.0)
                continue;
            double tau = sqrt(q) / L->dt;
            if (fabs(tau - (L->nt - 1)) < margin)
                margin = fabs(tau - (L->nt - 1));
            if (tau > (double)(L->nt - 1))
                continue;
            int64_t n = (int64_t)floor(tau);
            double f = tau - (double)n;
            M += 1;
            for (int k = -w; k <= w; ++k) {
                double aik = (1.0 - f) * sample_at(L, i, n + k) + f * sample_at(L, i, n + k + 1);
                s[k + w] += aik;
                E += aik * aik;
            }
        }
    }
    double N = 0.0;
    for (int k = 0; k < W; ++k)
        N += s[k] * s[k];
    double S = (M > 0 && E > 0.0) ? N / ((double)M * E) : 0.0;

    if (tau_l1)
        *tau_l1 = 0.0;
    if (grad) {
        for (int d = 0; d < P; ++d)
            grad[d] = 0.0;
        if (M > 0 && E > 0.0) {
            double coef = 2.0 / ((double)M * E);
            for (int32_t c = c_lo; c <= c_hi; ++c) {
                double dm = (double)(c - j) * L->dx;
                for (int64_t i = L->cmp_ptr[c]; i < L->cmp_ptr[c + 1]; ++i) {
                    double dq[3];
                    double q = traveltime_sq(L, p, t0, dm, L->offset[i], dq);
                    if (q <= 0.0)
                        continue;
                    double t = sqrt(q);
                    double tau = t / L->dt;
                    if (tau > (double)(L->nt - 1))
                        continue;
                    int64_t n = (int64_t)floor(tau);
                    double f = tau - (double)n;
                    double dS_dtau = 0.0;
                    for (int k = -w; k <= w; ++k) {
                        double u0 = sample_at(L, i, n + k), u1 = sample_at(L, i, n + k + 1);
                        double aik = (1.0 - f) * u0 + f * u1;
                        dS_dtau += coef * (s[k + w] - (double)M * S * aik) * (u1 - u0);
                    }
                    for (int d = 0; d < P; ++d)
                        grad[d] += dS_dtau * dq[d] / (2.0 * t * L->dt);
                    if (tau_l1)
                        *tau_l1 += fabs(dS_dtau);
                }
            }
        }
    }
    free(s);
    if (M_out)
        *M_out = M;
    if (margin_out)
        *margin_out = margin;
    return S;
}

double or_semblance(const or_line *L, int32_t j, int32_t n0, const double *p, int32_t *M_out,
                    double *margin_out)
{
    return semblance_impl(L, j, n0, p, M_out, margin_out, NULL, NULL);
}

double or_semblance_grad(const or_line *L, int32_t j, int32_t n0, const double *p, double *g)
{
    return semblance_impl(L, j, n0, p, NULL, NULL, g, NULL);
}

void or_semblance_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                        const double *params, double *S, int32_t *M, double *margin)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n; ++c) {
        int32_t m = 0;
        double mg = 0.0;
        S[c] = or_semblance(L, cmp[c], t[c], params + c * P, &m, &mg);
        if (M)
            M[c] = m;
        if (margin)
            margin[c] = mg;
    }
}

void or_semblance_grad_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                             const double *params, double *S, double *grad)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n; ++c)
        S[c] = or_semblance_grad(L, cmp[c], t[c], params + c * P, grad + c * P);
}

void or_semblance_tau_l1_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                               const double *params, double *l1)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n; ++c) {
        double g[3];
        semblance_impl(L, cmp[c], t[c], params + c * P, NULL, NULL, g, l1 + c);
    }
}

void or_kink_margin_batch(const or_line *L, int64_t n, const int32_t *cmp, const int32_t *t,
                          const double *params, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < n; ++c) {
        const int32_t j = cmp[c], n0 = t[c];
        const int32_t a = or_aperture(L, n0);
        const int32_t c_lo = j - a < 0 ? 0 : j - a;
        const int32_t c_hi = j + a > L->n_cmp - 1 ? L->n_cmp - 1 : j + a;
        const double t0 = (double)n0 * L->dt;
        const double *p = params + c * L->op;
        double m = INFINITY;
        for (int32_t cc = c_lo; cc <= c_hi; ++cc) {
            double dm = (double)(cc - j) * L->dx;
            for (int64_t i = L->cmp_ptr[cc]; i < L->cmp_ptr[cc + 1]; ++i) {
                double q = traveltime_sq(L, p, t0, dm, L->offset[i], NULL);
                if (q < 0.0)
                    continue;
                double tau = sqrt(q) / L->dt;
                if (tau > (double)(L->nt - 1))
                    continue;
                double d = fabs(tau - floor(tau + 0.5)) / (1.0 + fabs(tau - (double)n0));
                if (d < m)
                    m = d;
            }
        }
        out[c] = m;
    }
}
