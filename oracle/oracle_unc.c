/*
 * FP64 oracle: uncertainties of the fitted parameters at the optimum (Sec. 6).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Sec. 6 estimates the gradient of the merit function (the chi-square of
 * Sec. 5) at the optimum by finite differences whose steps come from the
 * spread of the final population about the optimum, sharpens those
 * derivatives by Richardson extrapolation to zero step within Neville's
 * algorithm, takes the Hessian H as the Jacobian of the resulting gradient,
 * and sets the variance of parameter j to [H^-1]_jj chi2(p_opt) / M.
 *
 * Derivative of one component (Ridders' extrapolation, as Press et al.
 * present it): central differences D_k = (F(x + t_k) - F(x - t_k)) / (2 t_k)
 * at t_k = h / C^k (C = 1.4, k < 10) have an error series in t_k^2, so the
 * Neville tableau T[k][0] = D_k, T[k][m] = (C^2m T[k][m-1] - T[k-1][m-1]) /
 * (C^2m - 1) extrapolates to t = 0.  The error of an entry is estimated as
 * its larger difference to its two parents; the result is the entry of
 * smallest estimated error; the tableau stops after the row whose diagonal
 * entry differs from the previous diagonal entry by at least twice that
 * error.
 *
 * Gradient: one such tableau per parameter i, F(t) = f(q + t e_i), initial
 * step h_i.  Hessian column j: one tableau per gradient component i on the
 * shared evaluations g(p + t e_j) and g(p - t e_j) (initial step h_j; a
 * component stops by its own rule, the column when every component has
 * stopped); H is then symmetrised, (H + H^T) / 2.
 *
 * Steps (readings of the paper's "spread around the identified optimum"):
 * oracle_population_steps gives h_j = the root-mean-square deviation from
 * p_opt of parameter j over the best quarter of the final population (at
 * least two individuals; fitness order, NaN last, ties to the lower index).
 * oracle_uncertainty then bounds each step to [1e-4, 0.1] (hi_j - lo_j) and
 * to half the distance from p_opt_j to the nearer bound, so every point of
 * the nested stencil (offsets up to 2 h_j) lies in the box; a parameter whose
 * bound leaves less than 1e-4 (hi_j - lo_j) of room is at the bound and is
 * held.  M is the number of free parameters.  Output per parameter: NaN if
 * it is held (not free, or at its bound); +infinity if H_jj = 0 (the merit
 * function does not depend on it), leaving it out of the inverse; NaN for
 * every parameter when the remaining H is not positive definite.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

double oracle__chi2_single(const double *par, double mu, const oracle_line *lines, int nlines,
                           const double *obs, const double *sigma, double *scratch);
int oracle__total_samples(const oracle_line *lines, int nlines);

#define NP ORACLE_NPAR
#define RID_C 1.4
#define RID_NTAB 10
#define RID_SAFE 2.0

/* Ridders tableaux for n components sharing one step sequence t_k = h / C^k.
 * diff(t, out, ctx) writes the n central differences at step t (components
 * with live[i] == 0 may be skipped by the callee).  best/err [n] receive the
 * estimates. */
typedef void (*diff_fn)(double t, const int *live, double *out, void *ctx);

static void ridders(int n, const int *act, double h, diff_fn diff, void *ctx, double *best,
                    double *err)
{
    double prev[RID_NTAB][NP], cur[RID_NTAB][NP], d[NP];
    int live[NP];
    int nlive = 0;
    for (int i = 0; i < n; ++i) {
        live[i] = act[i];
        nlive += live[i];
        best[i] = NAN;
        err[i] = HUGE_VAL;
    }
    double t = h;
    for (int k = 0; k < RID_NTAB && nlive > 0; ++k, t /= RID_C) {
        diff(t, live, d, ctx);
        for (int i = 0; i < n; ++i) {
            if (!live[i])
                continue;
            cur[0][i] = d[i];
            if (k == 0) {
                best[i] = d[i];
                continue;
            }
            double fac = RID_C * RID_C;
            for (int m = 1; m <= k; ++m, fac *= RID_C * RID_C) {
                cur[m][i] = (cur[m - 1][i] * fac - prev[m - 1][i]) / (fac - 1.0);
                const double e = fmax(fabs(cur[m][i] - cur[m - 1][i]),
                                      fabs(cur[m][i] - prev[m - 1][i]));
                if (e <= err[i]) {
                    err[i] = e;
                    best[i] = cur[m][i];
                }
            }
            if (fabs(cur[k][i] - prev[k - 1][i]) >= RID_SAFE * err[i]) {
                live[i] = 0;
                --nlive;
            }
        }
        for (int m = 0; m <= k; ++m)
            for (int i = 0; i < n; ++i)
                prev[m][i] = cur[m][i];
    }
}

typedef double (*obj_fn)(const double *p, void *ctx);

/* ---- gradient: one scalar tableau per parameter ------------------------- */

typedef struct {
    obj_fn f;
    void *ctx;
    const double *q;
    int n, i;
} grad_ctx;

static void grad_diff(double t, const int *live, double *out, void *c)
{
    const grad_ctx *g = (const grad_ctx *)c;
    (void)live;
    double a[NP], b[NP];
    memcpy(a, g->q, sizeof(double) * g->n);
    memcpy(b, g->q, sizeof(double) * g->n);
    a[g->i] += t;
    b[g->i] -= t;
    out[0] = (g->f(a, g->ctx) - g->f(b, g->ctx)) / (2.0 * t);
}

static void gradient(obj_fn f, void *ctx, int n, const double *q, const double *h,
                     const int *act, double *g, double *gerr)
{
    for (int i = 0; i < n; ++i) {
        g[i] = 0.0;
        gerr[i] = 0.0;
        if (!act[i])
            continue;
        grad_ctx c = {f, ctx, q, n, i};
        const int one = 1;
        ridders(1, &one, h[i], grad_diff, &c, &g[i], &gerr[i]);
    }
}

/* ---- Hessian: the Jacobian of that gradient ---------------------------- */

typedef struct {
    obj_fn f;
    void *ctx;
    int n;
    const double *p, *h;
    const int *act;
    int j;
} hess_ctx;

/* components whose tableau has stopped need no more gradient entries */
static void hess_diff(double t, const int *live, double *out, void *c)
{
    const hess_ctx *H = (const hess_ctx *)c;
    double a[NP], b[NP], ga[NP], gb[NP], ea[NP], eb[NP];
    memcpy(a, H->p, sizeof(double) * H->n);
    memcpy(b, H->p, sizeof(double) * H->n);
    a[H->j] += t;
    b[H->j] -= t;
    gradient(H->f, H->ctx, H->n, a, H->h, live, ga, ea);
    gradient(H->f, H->ctx, H->n, b, H->h, live, gb, eb);
    for (int i = 0; i < H->n; ++i)
        out[i] = (ga[i] - gb[i]) / (2.0 * t);
}

static void hessian(obj_fn f, void *ctx, int n, const double *p, const double *h,
                    const int *act, double *Hm, double *Herr)
{
    for (int j = 0; j < n; ++j) {
        double col[NP], cerr[NP];
        for (int i = 0; i < n; ++i) {
            col[i] = 0.0;
            cerr[i] = 0.0;
        }
        if (act[j]) {
            hess_ctx c = {f, ctx, n, p, h, act, j};
            ridders(n, act, h[j], hess_diff, &c, col, cerr);
        }
        for (int i = 0; i < n; ++i) {
            Hm[i * n + j] = act[i] ? col[i] : 0.0;
            if (Herr)
                Herr[i * n + j] = act[i] ? cerr[i] : 0.0;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double s = 0.5 * (Hm[i * n + j] + Hm[j * n + i]);
            Hm[i * n + j] = Hm[j * n + i] = s;
            if (Herr) {
                const double e = 0.5 * (Herr[i * n + j] + Herr[j * n + i]);
                Herr[i * n + j] = Herr[j * n + i] = e;
            }
        }
}

/* Exported for the pins: the Hessian of any objective (n <= 9), with the
 * same tableaux.  active [n] (may be NULL: all). */
int oracle_sec6_hessian(double (*f)(const double *, void *), void *ctx, int n, const double *p,
                        const double *h, const int32_t *active, double *Hm, double *Herr)
{
    if (n < 1 || n > NP)
        return -1;
    int act[NP];
    for (int i = 0; i < n; ++i)
        act[i] = active ? active[i] != 0 : 1;
    hessian(f, ctx, n, p, h, act, Hm, Herr);
    return 0;
}

/* sigma_j^2 = [H^-1]_jj c / M over the active parameters with H_jj != 0 */
static void sigmas_from(const double *Hm, const int *act, double c, int M, double *out)
{
    int keep[NP], idx[NP], m = 0;
    for (int j = 0; j < NP; ++j) {
        keep[j] = act[j] && Hm[j * NP + j] != 0.0;
        out[j] = !act[j] ? NAN : (keep[j] ? 0.0 : INFINITY);
        if (keep[j])
            idx[m++] = j;
    }
    if (m == 0)
        return;
    /* Cholesky of the kept block, then the diagonal of its inverse */
    double Lm[NP][NP];
    memset(Lm, 0, sizeof Lm);
    for (int a = 0; a < m; ++a)
        for (int b = 0; b <= a; ++b) {
            double s = Hm[idx[a] * NP + idx[b]];
            for (int k = 0; k < b; ++k)
                s -= Lm[a][k] * Lm[b][k];
            if (a == b) {
                if (!(s > 0.0)) {
                    for (int j = 0; j < NP; ++j)
                        out[j] = NAN;
                    return;
                }
                Lm[a][a] = sqrt(s);
            } else {
                Lm[a][b] = s / Lm[b][b];
            }
        }
    for (int r = 0; r < m; ++r) {
        /* solve H y = e_r; [H^-1]_rr = y_r */
        double y[NP], z[NP];
        for (int a = 0; a < m; ++a) {
            double s = a == r ? 1.0 : 0.0;
            for (int k = 0; k < a; ++k)
                s -= Lm[a][k] * z[k];
            z[a] = s / Lm[a][a];
        }
        for (int a = m - 1; a >= 0; --a) {
            double s = z[a];
            for (int k = a + 1; k < m; ++k)
                s -= Lm[k][a] * y[k];
            y[a] = s / Lm[a][a];
        }
        out[idx[r]] = sqrt(y[r] * c / (double)M);
    }
}

int oracle_sec6_sigmas(const double *Hm, const int32_t *active, double chi2, int M, double *out)
{
    int act[NP];
    for (int j = 0; j < NP; ++j)
        act[j] = active[j] != 0;
    if (M < 1)
        return -1;
    sigmas_from(Hm, act, chi2, M, out);
    return 0;
}

/* ---- the merit function of one pixel ----------------------------------- */

typedef struct {
    double mu;
    const oracle_line *lines;
    int nlines;
    const double *obs, *sigma;
    double *scratch;
} pix_ctx;

static double pix_chi2(const double *p, void *c)
{
    const pix_ctx *x = (const pix_ctx *)c;
    return oracle__chi2_single(p, x->mu, x->lines, x->nlines, x->obs, x->sigma, x->scratch);
}

static int popcount9(uint32_t m)
{
    int n = 0;
    for (int j = 0; j < NP; ++j)
        n += (m >> j) & 1u;
    return n;
}

int oracle_uncertainty(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const oracle_line *lines, int nlines, const double *lo, const double *hi,
                       const double *p_opt, const double *steps, uint32_t free_mask,
                       double *sigma_out, double *hess, double *hess_err, double *steps_used)
{
    for (int j = 0; j < NP; ++j)
        if (!(hi[j] > lo[j]))
            return -1;
    const int M = popcount9(free_mask & 0x1ffu);
    if (M < 1)
        return -1;
    const int L = oracle__total_samples(lines, nlines);
#pragma omp parallel
    {
        double *scratch = (double *)malloc(sizeof(double) * 4 * (size_t)L);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p) {
            const double *o = obs + p * 4 * L;
            const double *s = sigma + p * 4;
            const double *q = p_opt + p * NP;
            double *so = sigma_out + p * NP;
            int bad = 0;
            for (int i = 0; i < 4 * L; ++i)
                bad |= !isfinite(o[i]);
            for (int i = 0; i < 4; ++i)
                bad |= !(isfinite(s[i]) && s[i] > 0.0);
            for (int j = 0; j < NP; ++j)
                bad |= !isfinite(q[j]);
            double h[NP], Hm[NP * NP], He[NP * NP];
            int act[NP];
            for (int j = 0; j < NP; ++j) {
                const double span = hi[j] - lo[j];
                const double room = fmin(q[j] - lo[j], hi[j] - q[j]);
                double hj = steps[p * NP + j];
                if (!(hj >= 1e-4 * span))   /* also NaN */
                    hj = 1e-4 * span;
                if (hj > 0.1 * span)
                    hj = 0.1 * span;
                if (hj > 0.5 * room)
                    hj = 0.5 * room;
                act[j] = ((free_mask >> j) & 1u) && room >= 1e-4 * span;
                h[j] = act[j] ? hj : 0.0;
            }
            if (steps_used)
                memcpy(steps_used + p * NP, h, sizeof h);
            if (bad) {
                for (int j = 0; j < NP; ++j)
                    so[j] = NAN;
                if (hess)
                    for (int k = 0; k < NP * NP; ++k)
                        hess[p * NP * NP + k] = NAN;
                if (hess_err)
                    for (int k = 0; k < NP * NP; ++k)
                        hess_err[p * NP * NP + k] = NAN;
                continue;
            }
            pix_ctx c = {mu ? mu[p] : 1.0, lines, nlines, o, s, scratch};
            hessian(pix_chi2, &c, NP, q, h, act, Hm, He);
            sigmas_from(Hm, act, pix_chi2(q, &c), M, so);
            if (hess)
                memcpy(hess + p * NP * NP, Hm, sizeof Hm);
            if (hess_err)
                memcpy(hess_err + p * NP * NP, He, sizeof He);
        }
        free(scratch);
    }
    return 0;
}

/* ---- steps from the final population ------------------------------------ */

/* a before b in fitness order: smaller first, NaN last, ties to the lower index */
static int fit_before(double fa, int a, double fb, int b)
{
    const int na = isnan(fa), nb = isnan(fb);
    if (na != nb)
        return nb;
    if (!na && fa != fb)
        return fa < fb;
    return a < b;
}

int oracle_population_steps(const uint16_t *genes, const double *fitness, int64_t npix, int pop,
                            const double *lo, const double *hi, const double *p_opt,
                            double *steps)
{
    if (pop < 1)
        return -1;
    const int nb = pop < 2 ? pop : (pop / 4 > 2 ? pop / 4 : 2);
    for (int64_t p = 0; p < npix; ++p) {
        const double *f = fitness + p * pop;
        double acc[NP] = {0};
        for (int r = 0; r < nb; ++r) {
            /* the individual of rank r: the one with exactly r others before it */
            int who = -1;
            for (int i = 0; i < pop && who < 0; ++i) {
                int before = 0;
                for (int k = 0; k < pop; ++k)
                    before += k != i && fit_before(f[k], k, f[i], i);
                if (before == r)
                    who = i;
            }
            double par[NP];
            oracle_decode(genes + ((size_t)p * pop + who) * NP, lo, hi, par);
            for (int j = 0; j < NP; ++j) {
                const double d = par[j] - p_opt[p * NP + j];
                acc[j] += d * d;
            }
        }
        for (int j = 0; j < NP; ++j)
            steps[p * NP + j] = sqrt(acc[j] / nb);
    }
    return 0;
}
