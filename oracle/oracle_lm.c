/*
 * FP64 oracle: Levenberg-Marquardt refinement of one Milne-Eddington model
 * per pixel (the non-linear least-squares machinery of Sec. 5.3, applied to
 * the full model as the final polish of the genetic algorithm's best
 * individual; chi-square of Sec. 5).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Algorithm, in the normalised coordinates x_j = (p_j - lo_j)/(hi_j - lo_j)
 * kept inside [0, 1]:
 *   residuals r_i = (O_i - M_i(x)) / sigma_i over the 4L samples;
 *   Jacobian of the model by forward differences, step h = 1e-7 (taken
 *   backwards when x_j + h > 1): J_ij = (M_i(x + h e_j) - M_i(x)) / (h sigma_i),
 *   where for B, v_los, the Doppler width and the damping, which move every
 *   component's Faddeeva argument z = v + i a, M(x + h e_j) takes each
 *   component's w to first order about its value at x (oracle_me_synth_lin):
 *   one Faddeeva evaluation per component and sample serves all five models,
 *   and the difference from the exact model is of order |dz|^2, about h^2;
 *   A = J^T J, g = J^T r;
 *   trial: solve (A + lambda diag(A)) d = g by Cholesky (a parameter with
 *   A_jj = 0 gets d_j = 0), x' = clamp(x + d, 0, 1); accept if
 *   chi2(x') < chi2(x) (lambda /= 10, not below 1e-12), else lambda *= 10
 *   (not above 1e12) and retry, at most 10 trials per iteration; stop when a
 *   whole iteration fails.  lambda starts at 1e-3.
 *
 * A parameter outside free_mask (bit j = parameter j) is held: its Jacobian
 * column is zero, so it is treated like A_jj = 0 (d_j = 0).  The
 * non-magnetic pre-fit of Sec. 5.3 is this fit with B held
 * at 0 (the model then does not depend on the two field angles) and v_los,
 * the Doppler width, damping, eta0, S0 and S1 free.
 *
 * With the fill fraction of Sec. 5.2 (oracle_lm_fit_fill) the model is
 * alpha M(p) + (1 - alpha) I_c N e (oracle_fill.c) and alpha is a tenth
 * coordinate x_9 = (alpha - alpha_lo)/(alpha_hi - alpha_lo), fitted by the
 * same steps; nu = 4L - 10 in its chi-square.  The fit is the same algorithm
 * over 9 or 10 coordinates, so with alpha held at 1 it takes the steps of the
 * plain fit (the model is then M itself and only nu, which rescales every
 * chi-square alike, differs).
 *
 * The uncertainties of Sec. 6 at the result are computed separately
 * (oracle_unc.c).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

double oracle__chi2_single(const double *par, double mu, const oracle_line *lines, int nlines,
                           const double *obs, const double *sigma, double *scratch);
int oracle__total_samples(const oracle_line *lines, int nlines);

#define NP ORACLE_NPAR
#define MAXP (ORACLE_NPAR + 1)

/* One pixel's least-squares problem: the nine parameters, and with `fill`
 * the fill fraction as coordinate 9. */
typedef struct {
    int n;                         /* 9 or 10 coordinates */
    const double *lo, *hi;         /* [9] */
    double mu;
    const oracle_line *lines;
    int nlines;
    const oracle_fill *fill;       /* NULL: the plain model */
    const double *obs, *sigma;     /* [4L], [4] */
    int L;
} lm_problem;

static void to_params(const double *x, const double *lo, const double *hi, double *p)
{
    for (int j = 0; j < NP; ++j)
        p[j] = lo[j] + (hi[j] - lo[j]) * x[j];
}

static double to_alpha(const lm_problem *P, const double *x)
{
    return P->fill->alpha_lo + (P->fill->alpha_hi - P->fill->alpha_lo) * x[NP];
}

/* model [4L] at normalised x */
static void model_at(const lm_problem *P, const double *x, double *out)
{
    double p[NP];
    to_params(x, P->lo, P->hi, p);
    if (P->fill) {
        const double al = to_alpha(P, x);
        oracle_me_synth_fill(p, &al, 1, P->lines, P->nlines, &P->mu, P->fill, out);
    } else {
        oracle_me_synth(p, 1, P->lines, P->nlines, &P->mu, out);
    }
}

int oracle__fill_mix(const double *p, double alpha, double mu, const oracle_line *lines,
                     int nlines, const oracle_fill *fill, double *N, double *o);

/* model [4L] at normalised xs with every component's Faddeeva value taken to
 * first order about its value at x (the fill profile and fraction exact) */
static void model_lin(const lm_problem *P, const double *x, const double *xs, double *out)
{
    double p0[NP], p[NP];
    to_params(x, P->lo, P->hi, p0);
    to_params(xs, P->lo, P->hi, p);
    oracle_me_synth_lin(p0, p, P->mu, P->lines, P->nlines, out);
    if (P->fill) {
        double *N = (double *)malloc(sizeof(double) * P->L);
        oracle__fill_mix(p, to_alpha(P, xs), P->mu, P->lines, P->nlines, P->fill, N, out);
        free(N);
    }
}

/* coordinates that move the Faddeeva arguments: B, v_los, Doppler width, damping */
static int moves_profiles(int j)
{
    return j == 0 || j == 3 || j == 4 || j == 5;
}

static double chi2_at(const lm_problem *P, const double *x, double *scratch)
{
    double p[NP];
    to_params(x, P->lo, P->hi, p);
    if (!P->fill)
        return oracle__chi2_single(p, P->mu, P->lines, P->nlines, P->obs, P->sigma, scratch);
    /* Sec. 5 merit function of the fill model at this alpha */
    model_at(P, x, scratch);
    double c = 0.0;
    for (int s = 0; s < 4; ++s) {
        const double w2 = 1.0 / (P->sigma[s] * P->sigma[s]);
        for (int j = 0; j < P->L; ++j) {
            const double r = P->obs[s * P->L + j] - scratch[s * P->L + j];
            c += w2 * r * r;
        }
    }
    return c / (4.0 * P->L - 10.0);
}

/* J (R x n, normalised coordinates, weighted), A = J^T J and g = J^T r at x */
static void normal_equations(const lm_problem *P, const double *x, uint32_t free_mask,
                             double *m0, double *m1, double *J, double *A, double *g)
{
    const int n = P->n, L = P->L, R = 4 * L;
    const double *o = P->obs, *s = P->sigma;
    const double h = 1e-7;
    model_at(P, x, m0);
    for (int j = 0; j < n; ++j) {
        if (!((free_mask >> j) & 1u)) {
            for (int i = 0; i < R; ++i)
                J[i * n + j] = 0.0;
            continue;
        }
        double xs[MAXP];
        memcpy(xs, x, sizeof(double) * n);
        const double hj = (x[j] + h <= 1.0) ? h : -h;
        xs[j] += hj;
        if (moves_profiles(j))
            model_lin(P, x, xs, m1);
        else
            model_at(P, xs, m1);
        for (int i = 0; i < R; ++i)
            J[i * n + j] = (m1[i] - m0[i]) / (hj * s[i / L]);
    }
    for (int a = 0; a < n; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < n; ++b)
            A[a * n + b] = 0.0;
    }
    for (int i = 0; i < R; ++i) {
        const double r = (o[i] - m0[i]) / s[i / L];
        for (int a = 0; a < n; ++a) {
            g[a] += J[i * n + a] * r;
            for (int b = 0; b < n; ++b)
                A[a * n + b] += J[i * n + a] * J[i * n + b];
        }
    }
}

/* Cholesky solve of the SPD system M d = g (n x n, row-major, overwritten) */
static int cholesky_solve(int n, double *M, const double *g, double *d)
{
    double Lm[MAXP * MAXP];
    memset(Lm, 0, sizeof Lm);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = M[i * n + j];
            for (int k = 0; k < j; ++k)
                s -= Lm[i * n + k] * Lm[j * n + k];
            if (i == j) {
                if (!(s > 0.0))
                    return -1;
                Lm[i * n + i] = sqrt(s);
            } else {
                Lm[i * n + j] = s / Lm[j * n + j];
            }
        }
    }
    double y[MAXP];
    for (int i = 0; i < n; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k)
            s -= Lm[i * n + k] * y[k];
        y[i] = s / Lm[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k)
            s -= Lm[k * n + i] * d[k];
        d[i] = s / Lm[i * n + i];
    }
    return 0;
}

/* The damped iterations of one pixel from x (updated in place); returns the
 * iterations done, *c the chi-square at the result. */
static int lm_pixel(const lm_problem *P, double *x, int iterations, uint32_t free_mask, double *m0,
                    double *m1, double *J, double *scratch, double *c_out)
{
    const int n = P->n;
    double c = chi2_at(P, x, scratch);
    double lam = 1e-3;
    int it = 0;
    for (; it < iterations; ++it) {
        double A[MAXP * MAXP], g[MAXP];
        normal_equations(P, x, free_mask, m0, m1, J, A, g);
        int accepted = 0;
        for (int trial = 0; trial < 10 && !accepted; ++trial) {
            double M[MAXP * MAXP], gg[MAXP], d[MAXP];
            for (int a = 0; a < n; ++a) {
                for (int b = 0; b < n; ++b)
                    M[a * n + b] = A[a * n + b];
                gg[a] = g[a];
                if (A[a * n + a] == 0.0) {
                    for (int b = 0; b < n; ++b)
                        M[a * n + b] = M[b * n + a] = 0.0;
                    M[a * n + a] = 1.0;
                    gg[a] = 0.0;
                } else {
                    M[a * n + a] += lam * A[a * n + a];
                }
            }
            if (cholesky_solve(n, M, gg, d) != 0) {
                lam = lam * 10.0 > 1e12 ? 1e12 : lam * 10.0;
                continue;
            }
            double xn[MAXP];
            for (int j = 0; j < n; ++j) {
                const double v = x[j] + d[j];
                xn[j] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
            const double cn = chi2_at(P, xn, scratch);
            if (cn < c) {
                memcpy(x, xn, sizeof(double) * n);
                c = cn;
                lam = lam / 10.0 < 1e-12 ? 1e-12 : lam / 10.0;
                accepted = 1;
            } else {
                lam = lam * 10.0 > 1e12 ? 1e12 : lam * 10.0;
            }
        }
        if (!accepted)
            break;
    }
    *c_out = c;
    return it;
}

/* Both fits: the pixel loop; alpha_in / alpha_out only with fill. */
static int lm_fit_common(const double *obs, const double *sigma, const double *mu, int64_t npix,
                         const oracle_line *lines, int nlines, const double *lo,
                         const double *hi, const oracle_fill *fill, const double *params_in,
                         const double *alpha_in, int iterations, uint32_t free_mask,
                         double *params_out, double *alpha_out, double *chi2_out,
                         int32_t *iters_done)
{
    if (iterations < 0)
        return -1;
    for (int j = 0; j < NP; ++j)
        if (!(hi[j] > lo[j]))
            return -1;
    if (fill && !(fill->alpha_hi > fill->alpha_lo))
        return -1;
    const int n = fill ? NP + 1 : NP;
    const int L = oracle__total_samples(lines, nlines);
    const int R = 4 * L;
#pragma omp parallel
    {
        double *m0 = (double *)malloc(sizeof(double) * R);
        double *m1 = (double *)malloc(sizeof(double) * R);
        double *J = (double *)malloc(sizeof(double) * R * n);
        double *scratch = (double *)malloc(sizeof(double) * R);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p) {
            lm_problem P = {n, lo, hi, mu ? mu[p] : 1.0, lines, nlines, fill,
                            obs + p * R, sigma + p * 4, L};
            int bad = 0;
            for (int i = 0; i < R; ++i)
                if (!isfinite(P.obs[i]))
                    bad = 1;
            for (int i = 0; i < 4; ++i)
                if (!(isfinite(P.sigma[i]) && P.sigma[i] > 0.0))
                    bad = 1;
            if (fill && !bad) {
                /* a field-free profile that is invalid at this mu */
                double *N = scratch;
                for (int l = 0, off = 0; l < nlines; off += lines[l].nlam, ++l)
                    if (oracle_fill_profile(&lines[l], &fill->line[l], P.mu,
                                            params_in[p * NP + 3], N + off) != 0)
                        bad = 1;
            }
            double x[MAXP];
            for (int j = 0; j < NP; ++j) {
                double v = (params_in[p * NP + j] - lo[j]) / (hi[j] - lo[j]);
                x[j] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
            if (fill) {
                double v = (alpha_in[p] - fill->alpha_lo) / (fill->alpha_hi - fill->alpha_lo);
                x[NP] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
            if (bad) {
                for (int j = 0; j < NP; ++j)
                    params_out[p * NP + j] = NAN;
                if (fill)
                    alpha_out[p] = NAN;
                chi2_out[p] = NAN;
                if (iters_done)
                    iters_done[p] = 0;
                continue;
            }
            double c;
            const int it = lm_pixel(&P, x, iterations, free_mask, m0, m1, J, scratch, &c);
            to_params(x, lo, hi, params_out + p * NP);
            if (fill)
                alpha_out[p] = to_alpha(&P, x);
            chi2_out[p] = c;
            if (iters_done)
                iters_done[p] = it;
        }
        free(m0);
        free(m1);
        free(J);
        free(scratch);
    }
    return 0;
}

int oracle_lm_refine(const double *obs, const double *sigma, const double *mu, int64_t npix,
                     const oracle_line *lines, int nlines, const double *lo, const double *hi,
                     const double *params_in, int iterations, double *params_out,
                     double *chi2_out, int32_t *iters_done)
{
    return oracle_lm_fit(obs, sigma, mu, npix, lines, nlines, lo, hi, params_in, iterations,
                         0x1ffu, params_out, chi2_out, iters_done);
}

int oracle_lm_fit(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const oracle_line *lines, int nlines, const double *lo, const double *hi,
                  const double *params_in, int iterations, uint32_t free_mask,
                  double *params_out, double *chi2_out, int32_t *iters_done)
{
    return lm_fit_common(obs, sigma, mu, npix, lines, nlines, lo, hi, NULL, params_in, NULL,
                         iterations, free_mask & 0x1ffu, params_out, NULL, chi2_out,
                         iters_done);
}

int oracle_lm_fit_fill(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const oracle_line *lines, int nlines, const double *lo, const double *hi,
                       const oracle_fill *fill, const double *params_in, const double *alpha_in,
                       int iterations, uint32_t free_mask, double *params_out,
                       double *alpha_out, double *chi2_out, int32_t *iters_done)
{
    if (!fill || !alpha_in || !alpha_out)
        return -1;
    return lm_fit_common(obs, sigma, mu, npix, lines, nlines, lo, hi, fill, params_in, alpha_in,
                         iterations, free_mask & 0x3ffu, params_out, alpha_out, chi2_out,
                         iters_done);
}
