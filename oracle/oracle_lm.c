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
 *   backwards when x_j + h > 1): J_ij = (M_i(x + h e_j) - M_i(x)) / (h sigma_i);
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

static void to_params(const double *x, const double *lo, const double *hi, double *p)
{
    for (int j = 0; j < NP; ++j)
        p[j] = lo[j] + (hi[j] - lo[j]) * x[j];
}

/* model [4L] at normalised x */
static void model_at(const double *x, const double *lo, const double *hi, double mu,
                     const oracle_line *lines, int nlines, double *out)
{
    double p[NP];
    to_params(x, lo, hi, p);
    oracle_me_synth(p, 1, lines, nlines, &mu, out);
}

static double chi2_at(const double *x, const double *lo, const double *hi, double mu,
                      const oracle_line *lines, int nlines, const double *obs,
                      const double *sigma, double *scratch)
{
    double p[NP];
    to_params(x, lo, hi, p);
    return oracle__chi2_single(p, mu, lines, nlines, obs, sigma, scratch);
}

/* J (R x 9, normalised coordinates, weighted), A = J^T J and g = J^T r at x */
static void normal_equations(const double *x, const double *lo, const double *hi, double mu,
                             const oracle_line *lines, int nlines, const double *o,
                             const double *s, int L, uint32_t free_mask, double *m0,
                             double *m1, double *J, double *A, double *g)
{
    const int R = 4 * L;
    const double h = 1e-7;
    model_at(x, lo, hi, mu, lines, nlines, m0);
    for (int j = 0; j < NP; ++j) {
        if (!((free_mask >> j) & 1u)) {
            for (int i = 0; i < R; ++i)
                J[i * NP + j] = 0.0;
            continue;
        }
        double xs[NP];
        memcpy(xs, x, sizeof xs);
        const double hj = (x[j] + h <= 1.0) ? h : -h;
        xs[j] += hj;
        model_at(xs, lo, hi, mu, lines, nlines, m1);
        for (int i = 0; i < R; ++i)
            J[i * NP + j] = (m1[i] - m0[i]) / (hj * s[i / L]);
    }
    for (int a = 0; a < NP; ++a) {
        g[a] = 0.0;
        for (int b = 0; b < NP; ++b)
            A[a * NP + b] = 0.0;
    }
    for (int i = 0; i < R; ++i) {
        const double r = (o[i] - m0[i]) / s[i / L];
        for (int a = 0; a < NP; ++a) {
            g[a] += J[i * NP + a] * r;
            for (int b = 0; b < NP; ++b)
                A[a * NP + b] += J[i * NP + a] * J[i * NP + b];
        }
    }
}

/* Cholesky solve of the SPD system M d = g (9 x 9, row-major, overwritten) */
static int cholesky_solve(double *M, const double *g, double *d)
{
    double Lm[NP * NP];
    memset(Lm, 0, sizeof Lm);
    for (int i = 0; i < NP; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = M[i * NP + j];
            for (int k = 0; k < j; ++k)
                s -= Lm[i * NP + k] * Lm[j * NP + k];
            if (i == j) {
                if (!(s > 0.0))
                    return -1;
                Lm[i * NP + i] = sqrt(s);
            } else {
                Lm[i * NP + j] = s / Lm[j * NP + j];
            }
        }
    }
    double y[NP];
    for (int i = 0; i < NP; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k)
            s -= Lm[i * NP + k] * y[k];
        y[i] = s / Lm[i * NP + i];
    }
    for (int i = NP - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < NP; ++k)
            s -= Lm[k * NP + i] * d[k];
        d[i] = s / Lm[i * NP + i];
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
    if (iterations < 0)
        return -1;
    for (int j = 0; j < NP; ++j)
        if (!(hi[j] > lo[j]))
            return -1;
    const int L = oracle__total_samples(lines, nlines);
    const int R = 4 * L;
#pragma omp parallel
    {
        double *m0 = (double *)malloc(sizeof(double) * R);
        double *m1 = (double *)malloc(sizeof(double) * R);
        double *J = (double *)malloc(sizeof(double) * R * NP);
        double *scratch = (double *)malloc(sizeof(double) * R);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p) {
            const double *o = obs + p * R;
            const double *s = sigma + p * 4;
            const double m = mu ? mu[p] : 1.0;
            int bad = 0;
            for (int i = 0; i < R; ++i)
                if (!isfinite(o[i]))
                    bad = 1;
            for (int i = 0; i < 4; ++i)
                if (!(isfinite(s[i]) && s[i] > 0.0))
                    bad = 1;
            double x[NP];
            for (int j = 0; j < NP; ++j) {
                double v = (params_in[p * NP + j] - lo[j]) / (hi[j] - lo[j]);
                x[j] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
            if (bad) {
                for (int j = 0; j < NP; ++j)
                    params_out[p * NP + j] = NAN;
                chi2_out[p] = NAN;
                if (iters_done)
                    iters_done[p] = 0;
                continue;
            }
            double c = chi2_at(x, lo, hi, m, lines, nlines, o, s, scratch);
            double lam = 1e-3;
            int it = 0;
            for (; it < iterations; ++it) {
                double A[NP * NP], g[NP];
                normal_equations(x, lo, hi, m, lines, nlines, o, s, L, free_mask, m0, m1, J, A, g);
                int accepted = 0;
                for (int trial = 0; trial < 10 && !accepted; ++trial) {
                    double M[NP * NP], gg[NP], d[NP];
                    for (int a = 0; a < NP; ++a) {
                        for (int b = 0; b < NP; ++b)
                            M[a * NP + b] = A[a * NP + b];
                        gg[a] = g[a];
                        if (A[a * NP + a] == 0.0) {
                            for (int b = 0; b < NP; ++b)
                                M[a * NP + b] = M[b * NP + a] = 0.0;
                            M[a * NP + a] = 1.0;
                            gg[a] = 0.0;
                        } else {
                            M[a * NP + a] += lam * A[a * NP + a];
                        }
                    }
                    if (cholesky_solve(M, gg, d) != 0) {
                        lam = lam * 10.0 > 1e12 ? 1e12 : lam * 10.0;
                        continue;
                    }
                    double xn[NP];
                    for (int j = 0; j < NP; ++j) {
                        const double v = x[j] + d[j];
                        xn[j] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
                    }
                    const double cn = chi2_at(xn, lo, hi, m, lines, nlines, o, s, scratch);
                    if (cn < c) {
                        memcpy(x, xn, sizeof x);
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
            to_params(x, lo, hi, params_out + p * NP);
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
