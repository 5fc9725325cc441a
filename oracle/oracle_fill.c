/*
 * FP64 oracle: magnetic fill fraction (Sec. 5.2).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * A fraction alpha of the pixel is magnetic and the rest field-free, so the
 * Stokes vector is
 *   alpha M(p) + (1 - alpha) I_c N(lambda) e,   e = (1, 0, 0, 0),
 * with M the Milne-Eddington vector of the nine parameters p, I_c = S0 + mu S1
 * its continuum and N the normalised Stokes I profile of the field-free
 * surroundings.  The paper parameterises N as a Voigt profile whose
 * amplitude, width and damping follow cubic polynomials in mu fitted to
 * measured centre-to-limb variations; those fits are not published, so the
 * coefficients are inputs here:
 *   N(lambda) = 1 - d(mu) H(v, a(mu)) / H(0, a(mu)),
 *   v = (lambda - lambda0 (1 + v_los / c)) / w(mu)   (centred on the model's
 *                                                     line centre),
 *   d, w, a = sum_{k=0..3} coef_k mu^k   (per line: depth, width [A], damping).
 * alpha enters linearly, so for given p the chi-square of Sec. 5 is a
 * quadratic in alpha.  Its minimiser over [alpha_lo, alpha_hi] is
 *   alpha* = clamp(sum w^2 (O - b) . D / sum w^2 D . D),
 *   b = I_c N e,  D = M - b   (alpha_hi when sum w^2 D . D = 0),
 * and the fitness is chi2(alpha*) = (1/nu) sum w^2 |O - b - alpha* D|^2 with
 * nu = 4L - 10 (alpha is a tenth fitted parameter).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle__total_samples(const oracle_line *lines, int nlines);

static double cubic(const double c[4], double mu)
{
    return c[0] + mu * (c[1] + mu * (c[2] + mu * c[3]));
}

int oracle_fill_profile(const oracle_line *ln, const oracle_fill_line *f, double mu, double vlos,
                        double *N)
{
    const double d = cubic(f->depth, mu), w = cubic(f->width, mu), a = cubic(f->damp, mu);
    if (!(isfinite(d) && isfinite(w) && isfinite(a) && w > 0.0 && a >= 0.0 && a <= 1.5))
        return -1;
    double h0, l0;
    oracle_faddeeva(0.0, a, &h0, &l0);
    const double lc = ln->lambda0 * (1.0 + vlos / ORACLE_C_KMS);
    for (int j = 0; j < ln->nlam; ++j) {
        const double v = (ln->start + ln->step * j - lc) / w;
        double h, l;
        oracle_faddeeva(fabs(v), a, &h, &l);
        N[j] = 1.0 - d * h / h0;
    }
    return 0;
}

/* N of every line, concatenated [L]; 0 or -1 */
static int fill_profiles(const oracle_line *lines, int nlines, const oracle_fill *fill, double mu,
                         double vlos, double *N)
{
    int off = 0;
    for (int l = 0; l < nlines; ++l) {
        if (oracle_fill_profile(&lines[l], &fill->line[l], mu, vlos, N + off) != 0)
            return -1;
        off += lines[l].nlam;
    }
    return 0;
}

/* o [4][L] holds M(p); replace it by alpha M(p) + (1 - alpha) I_c N e (NaN
 * and -1 where N is invalid).  N [L] is scratch. */
int oracle__fill_mix(const double *p, double alpha, double mu, const oracle_line *lines,
                     int nlines, const oracle_fill *fill, double *N, double *o)
{
    const int L = oracle__total_samples(lines, nlines);
    if (fill_profiles(lines, nlines, fill, mu, p[3], N) != 0) {
        for (int k = 0; k < 4 * L; ++k)
            o[k] = NAN;
        return -1;
    }
    const double ic = p[7] + mu * p[8];
    for (int j = 0; j < L; ++j)
        o[j] = alpha * o[j] + (1.0 - alpha) * ic * N[j];
    for (int k = L; k < 4 * L; ++k)
        o[k] *= alpha;
    return 0;
}

int oracle_me_synth_fill(const double *par, const double *alpha, int64_t n,
                         const oracle_line *lines, int nlines, const double *mu,
                         const oracle_fill *fill, double *out)
{
    const int L = oracle__total_samples(lines, nlines);
    double *N = (double *)malloc(sizeof(double) * L);
    int rc = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double *p = par + i * ORACLE_NPAR;
        double *o = out + i * 4 * L;
        oracle_me_synth(p, 1, lines, nlines, mu ? mu + i : NULL, o);
        if (oracle__fill_mix(p, alpha[i], mu ? mu[i] : 1.0, lines, nlines, fill, N, o) != 0)
            rc = -1;
    }
    free(N);
    return rc;
}

double oracle__chi2_fill_single(const double *par, double mu, const oracle_line *lines,
                                int nlines, const double *obs, const double *sigma,
                                const oracle_fill *fill, double *scratch, double *alpha_out)
{
    const int L = oracle__total_samples(lines, nlines);
    double *M = scratch, *N = scratch + 4 * L;
    oracle_me_synth(par, 1, lines, nlines, &mu, M);
    if (fill_profiles(lines, nlines, fill, mu, par[3], N) != 0) {
        *alpha_out = NAN;
        return NAN;
    }
    const double ic = par[7] + mu * par[8];
    double num = 0.0, den = 0.0;
    for (int s = 0; s < 4; ++s) {
        const double w2 = 1.0 / (sigma[s] * sigma[s]);
        for (int j = 0; j < L; ++j) {
            const double b = s == 0 ? ic * N[j] : 0.0;
            const double D = M[s * L + j] - b;
            num += w2 * (obs[s * L + j] - b) * D;
            den += w2 * D * D;
        }
    }
    double al = den > 0.0 ? num / den : fill->alpha_hi;
    al = al < fill->alpha_lo ? fill->alpha_lo : (al > fill->alpha_hi ? fill->alpha_hi : al);
    double c = 0.0;
    for (int s = 0; s < 4; ++s) {
        const double w2 = 1.0 / (sigma[s] * sigma[s]);
        for (int j = 0; j < L; ++j) {
            const double b = s == 0 ? ic * N[j] : 0.0;
            const double r = obs[s * L + j] - b - al * (M[s * L + j] - b);
            c += w2 * r * r;
        }
    }
    *alpha_out = al;
    return c / (4.0 * L - 10.0);
}

void oracle_chi2_fill(const double *par, int64_t npix, int pop, const oracle_line *lines,
                      int nlines, const double *obs, const double *sigma, const double *mu,
                      const oracle_fill *fill, double *chi2, double *alpha)
{
    const int L = oracle__total_samples(lines, nlines);
#pragma omp parallel
    {
        double *scratch = (double *)malloc(sizeof(double) * 5 * L);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p)
            for (int i = 0; i < pop; ++i)
                chi2[p * pop + i] = oracle__chi2_fill_single(
                    par + (p * pop + i) * ORACLE_NPAR, mu ? mu[p] : 1.0, lines, nlines,
                    obs + p * 4 * L, sigma + p * 4, fill, scratch, alpha + p * pop + i);
        free(scratch);
    }
}
