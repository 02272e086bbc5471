/*
 * Gradient polish and reference maxima of the semblance.  Test
 * infrastructure (see oracle.h).
 *
 * Neither is part of the paper's gradient-free method: the polish is a
 * differentiable refinement of each domain's winner, the reference maximum is
 * what the search result is measured against (the semblance gap).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Adam (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8) ascending S on the
 * box-normalised coordinates z = (p - lo) / (hi - lo), projected onto [0,1];
 * each step scores the new point and the best point seen is returned. */
void or_polish(const or_line *L, const or_bounds *B, int64_t n, const int32_t *cmp,
               const int32_t *t, const float *p_in, double lr, int32_t steps,
               double *p_out, double *S_out)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < n; ++c) {
        float lof[3], hif[3];
        or_sample_bounds(L, B, t[c], lof, hif);
        double lo[3], span[3], z[3], m[3] = {0, 0, 0}, v[3] = {0, 0, 0};
        double p[3] = {0, 0, 0}, best_p[3] = {0, 0, 0}, g[3];
        for (int d = 0; d < P; ++d) {
            lo[d] = lof[d];
            span[d] = (double)hif[d] - (double)lof[d];
            p[d] = p_in[c * P + d];
            best_p[d] = p[d];
            z[d] = (p[d] - lo[d]) / span[d];
        }
        double best_S = or_semblance(L, cmp[c], t[c], p, NULL, NULL);
        double b1k = 1.0, b2k = 1.0;
        for (int k = 1; k <= steps; ++k) {
            or_semblance_grad(L, cmp[c], t[c], p, g);
            b1k *= 0.9;
            b2k *= 0.999;
            for (int d = 0; d < P; ++d) {
                double gz = g[d] * span[d];
                m[d] = 0.9 * m[d] + 0.1 * gz;
                v[d] = 0.999 * v[d] + 0.001 * gz * gz;
                double mh = m[d] / (1.0 - b1k), vh = v[d] / (1.0 - b2k);
                z[d] += lr * mh / (sqrt(vh) + 1e-8);
                if (z[d] < 0.0)
                    z[d] = 0.0;
                if (z[d] > 1.0)
                    z[d] = 1.0;
                p[d] = lo[d] + z[d] * span[d];
            }
            double S = or_semblance(L, cmp[c], t[c], p, NULL, NULL);
            if (S > best_S) {
                best_S = S;
                memcpy(best_p, p, sizeof(p));
            }
        }
        for (int d = 0; d < P; ++d)
            p_out[c * P + d] = best_p[d];
        S_out[c] = best_S;
    }
}

/* ---------------------------------------------------------------------------
 * reference maximum: uniform grid over the sample's box, then Nelder-Mead
 * (reflection 1, expansion 2, contraction 1/2, shrink 1/2) in box-normalised
 * coordinates, clamped to the box, from the n_refine best grid points. */

typedef struct {
    const or_line *L;
    int32_t j, n0, P;
    double lo[3], span[3];
    double best_S, best_p[3];
} sref_ctx;

static double sref_eval(sref_ctx *c, const double *z)
{
    double p[3] = {0, 0, 0}, zz[3];
    for (int d = 0; d < c->P; ++d) {
        zz[d] = z[d] < 0.0 ? 0.0 : (z[d] > 1.0 ? 1.0 : z[d]);
        p[d] = c->lo[d] + zz[d] * c->span[d];
    }
    double S = or_semblance(c->L, c->j, c->n0, p, NULL, NULL);
    if (S > c->best_S) {
        c->best_S = S;
        memcpy(c->best_p, p, sizeof(p));
    }
    return S;
}

static void nelder_mead(sref_ctx *c, const double *z0, const double *step, int max_eval)
{
    const int P = c->P;
    double x[4][3], f[4];
    for (int i = 0; i <= P; ++i) {
        for (int d = 0; d < P; ++d)
            x[i][d] = z0[d];
        if (i > 0)
            x[i][i - 1] += step[i - 1];
        f[i] = -sref_eval(c, x[i]);
    }
    int evals = P + 1;
    while (evals < max_eval) {
        /* order: best first */
        for (int a = 0; a <= P; ++a)
            for (int b = a + 1; b <= P; ++b)
                if (f[b] < f[a]) {
                    double tf = f[a]; f[a] = f[b]; f[b] = tf;
                    for (int d = 0; d < P; ++d) {
                        double tx = x[a][d]; x[a][d] = x[b][d]; x[b][d] = tx;
                    }
                }
        double size = 0.0;
        for (int i = 1; i <= P; ++i)
            for (int d = 0; d < P; ++d)
                size = fmax(size, fabs(x[i][d] - x[0][d]));
        if (size < 1e-9)
            break;
        double cen[3] = {0, 0, 0}, xr[3], xe[3], xc[3];
        for (int i = 0; i < P; ++i)
            for (int d = 0; d < P; ++d)
                cen[d] += x[i][d] / P;
        for (int d = 0; d < P; ++d)
            xr[d] = cen[d] + (cen[d] - x[P][d]);
        double fr = -sref_eval(c, xr);
        ++evals;
        if (fr < f[0]) {
            for (int d = 0; d < P; ++d)
                xe[d] = cen[d] + 2.0 * (cen[d] - x[P][d]);
            double fe = -sref_eval(c, xe);
            ++evals;
            if (fe < fr) {
                memcpy(x[P], xe, sizeof(xe)); f[P] = fe;
            } else {
                memcpy(x[P], xr, sizeof(xr)); f[P] = fr;
            }
        } else if (fr < f[P - 1]) {
            memcpy(x[P], xr, sizeof(xr)); f[P] = fr;
        } else {
            for (int d = 0; d < P; ++d)
                xc[d] = cen[d] + 0.5 * (x[P][d] - cen[d]);
            double fc = -sref_eval(c, xc);
            ++evals;
            if (fc < f[P]) {
                memcpy(x[P], xc, sizeof(xc)); f[P] = fc;
            } else {
                for (int i = 1; i <= P; ++i) {
                    for (int d = 0; d < P; ++d)
                        x[i][d] = x[0][d] + 0.5 * (x[i][d] - x[0][d]);
                    f[i] = -sref_eval(c, x[i]);
                    ++evals;
                }
            }
        }
    }
}

void or_sref(const or_line *L, const or_bounds *B, int64_t n, const int32_t *cmp,
             const int32_t *t, const int32_t *grid, int32_t n_refine, double *S_ref,
             double *p_ref)
{
    const int P = L->op;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n; ++c) {
        sref_ctx sc;
        memset(&sc, 0, sizeof(sc));
        sc.L = L; sc.j = cmp[c]; sc.n0 = t[c]; sc.P = P; sc.best_S = -1.0;
        float lof[3], hif[3];
        or_sample_bounds(L, B, t[c], lof, hif);
        int ng[3] = {1, 1, 1};
        int64_t total = 1;
        for (int d = 0; d < P; ++d) {
            sc.lo[d] = lof[d];
            sc.span[d] = (double)hif[d] - (double)lof[d];
            ng[d] = grid[d] < 2 ? 2 : grid[d];
            total *= ng[d];
        }
        int nr = n_refine < 1 ? 1 : (n_refine > 16 ? 16 : n_refine);
        double top_S[16];
        double top_z[16][3];
        for (int r = 0; r < nr; ++r)
            top_S[r] = -1.0;
        for (int64_t g = 0; g < total; ++g) {
            double z[3] = {0, 0, 0};
            int64_t rem = g;
            for (int d = 0; d < P; ++d) {
                z[d] = (double)(rem % ng[d]) / (double)(ng[d] - 1);
                rem /= ng[d];
            }
            double S = sref_eval(&sc, z);
            /* keep the nr best grid points */
            int worst = 0;
            for (int r = 1; r < nr; ++r)
                if (top_S[r] < top_S[worst])
                    worst = r;
            if (S > top_S[worst]) {
                top_S[worst] = S;
                memcpy(top_z[worst], z, sizeof(z));
            }
        }
        double step[3];
        for (int d = 0; d < P; ++d)
            step[d] = 1.0 / (double)(ng[d] - 1);
        for (int r = 0; r < nr; ++r)
            if (top_S[r] >= 0.0)
                nelder_mead(&sc, top_z[r], step, 300);
        S_ref[c] = sc.best_S;
        for (int d = 0; d < P; ++d)
            p_ref[c * P + d] = sc.best_p[d];
    }
}
