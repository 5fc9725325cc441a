/*
 * The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * entry point driven once on small inputs (both Fe I 6302 lines, a bad
 * pixel, ragged populations), checking only that results are finite where
 * they must be; the numbers themselves are pinned by the Python tests.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static void make_line(oracle_line *ln, double lam0, double Jl, double gl, double Ju, double gu,
                      int nlam)
{
    memset(ln, 0, sizeof *ln);
    ln->lambda0 = lam0;
    ln->ncomp = oracle_zeeman(Jl, gl, Ju, gu, ln->q, ln->shift, ln->strength, ORACLE_MAXCOMP);
    ln->start = lam0 - 0.4;
    ln->step = 0.8 / (nlam - 1);
    ln->nlam = nlam;
}

static double quad(const double *p, void *ctx)
{
    (void)ctx;
    return 3.0 * p[0] * p[0] + p[0] * p[1] + 2.0 * p[1] * p[1] + p[2] * p[2] * p[2] * p[2];
}

int main(void)
{
    enum { NPIX = 3, POP = 12, NL = 2, NLAM = 24, L = NL * NLAM };
    oracle_line lines[NL];
    make_line(&lines[0], 6301.5091, 2, 11.0 / 6.0, 2, 1.5, NLAM);
    make_line(&lines[1], 6302.5017, 1, 2.5, 0, 0.0, NLAM);
    CHECK(lines[0].ncomp == 12 && lines[1].ncomp == 3);
    double re, im;
    oracle_faddeeva(1.3, 0.2, &re, &im);
    CHECK(isfinite(re) && isfinite(im));
    CHECK(oracle_lande_ls(2, 1, 2) > 1.8);
    CHECK(isfinite(oracle_wigner3j(1, 2, 1, 0, 1, -1)));

    const double lo[9] = {0, 0, 0, -7.5, 0.02, 0, 1, 0, 0.5};
    const double hi[9] = {3000, 180, 180, 7.5, 0.05, 0.5, 30, 0.5, 1};
    double truth[NPIX * 9];
    for (int p = 0; p < NPIX; ++p)
        for (int j = 0; j < 9; ++j)
            truth[p * 9 + j] = lo[j] + (hi[j] - lo[j]) * (0.2 + 0.25 * p + 0.03 * j);
    const double mu[NPIX] = {1.0, 0.8, 0.6};
    double *obs = malloc(sizeof(double) * NPIX * 4 * L);
    oracle_me_synth(truth, NPIX, lines, NL, mu, obs);
    double sigma[NPIX * 4];
    for (int p = 0; p < NPIX; ++p)
        for (int s = 0; s < 4; ++s)
            sigma[p * 4 + s] = 1e-3;
    obs[2 * 4 * L + 5] = NAN;  /* pixel 2 is bad */
    double chi[NPIX];
    oracle_chi2(truth, NPIX, 1, lines, NL, obs, sigma, mu, chi);
    CHECK(chi[0] < 1e-20 && isnan(chi[2]));

    /* random stream, operators */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out4[4];
    oracle_philox4x32_10(ctr, key, out4);
    uint16_t genes[POP * 9], genes2[POP * 9], masks[POP * 9];
    oracle_ga_init(7, 0, POP, 0, 0, 0, NULL, NULL, NULL, 0, genes);
    oracle_ga_init(7, 0, POP, 5, 300, 2, truth, lo, hi, 1, genes2);
    double par[POP * 9], fit[POP];
    for (int i = 0; i < POP; ++i) {
        oracle_decode(genes + i * 9, lo, hi, par + i * 9);
        fit[i] = (double)((i * 7) % 5);
    }
    fit[3] = NAN;
    int32_t parents[POP * 2], xpoint[POP], elite, replaced[POP];
    CHECK(oracle_ga_step(genes, fit, POP, 4, 0.85, 0.05, 7, 0, 1, genes2, parents, xpoint, masks,
                         &elite) == 0);
    CHECK(oracle_ga_step(genes, fit, POP, POP + 1, 0.85, 0.05, 7, 0, 1, genes2, parents, xpoint,
                         masks, &elite) != 0);
    uint32_t polys[16], pt[9], dirs[9][32];
    CHECK(oracle_sobol_polys(polys, 16) == 16);
    oracle_sobol_directions(dirs);
    oracle_sobol_point(12345u, pt);
    oracle_ga_restart(genes, fit, POP, 7, 0, 4, 4, genes2, replaced);

    /* the whole GA, plain and with fill fraction, seeded and boxed */
    double bp[NPIX * 9], bc[NPIX], ba[NPIX], ff[NPIX * POP];
    int32_t st[NPIX];
    uint16_t fg[NPIX * POP * 9];
    CHECK(oracle_ga_invert(obs, sigma, mu, NPIX, lines, NL, lo, hi, NULL, NULL, NULL, POP, 3, 4,
                           0.85, 0.05, 1, 0, 0, 0, 0, NULL, 1, 2, bp, bc, st, fg, ff) == 0);
    CHECK(st[0] == 0 && st[2] == 1 && isfinite(bc[0]) && isnan(bc[2]));
    oracle_fill fill;
    memset(&fill, 0, sizeof fill);
    fill.alpha_lo = 0.1;
    fill.alpha_hi = 1.0;
    for (int l = 0; l < NL; ++l) {
        fill.line[l].depth[0] = 0.6;
        fill.line[l].width[0] = 0.03;
        fill.line[l].damp[0] = 0.3;
    }
    double box[NPIX * 18];
    for (int p = 0; p < NPIX; ++p)
        for (int j = 0; j < 9; ++j) {
            box[p * 18 + j] = lo[j];
            box[p * 18 + 9 + j] = hi[j];
        }
    CHECK(oracle_ga_invert(obs, sigma, mu, NPIX, lines, NL, lo, hi, box, &fill, ba, POP, 2, 3,
                           0.85, 0.05, 2, 5, 3, 16, 1, truth, 0, 0, bp, bc, st, NULL, NULL) == 0);
    CHECK(isfinite(ba[0]) && isnan(ba[2]));
    double N[NLAM], ofill[NPIX * 4 * L], cf[NPIX * POP], af[NPIX * POP];
    CHECK(oracle_fill_profile(&lines[0], &fill.line[0], 0.9, 1.0, N) == 0);
    const double alpha[NPIX] = {0.5, 0.7, 0.9};
    CHECK(oracle_me_synth_fill(truth, alpha, NPIX, lines, NL, mu, &fill, ofill) == 0);
    oracle_chi2_fill(truth, NPIX, 1, lines, NL, obs, sigma, mu, &fill, cf, af);

    /* refinements, pre-fit form, uncertainties */
    double po[NPIX * 9], co[NPIX], ao[NPIX];
    int32_t it[NPIX];
    CHECK(oracle_lm_refine(obs, sigma, mu, NPIX, lines, NL, lo, hi, bp, 3, po, co, it) == 0);
    CHECK(oracle_lm_fit(obs, sigma, mu, NPIX, lines, NL, lo, hi, bp, 3, 0x1f8u, po, co, NULL) == 0);
    CHECK(oracle_lm_fit_fill(ofill, sigma, mu, NPIX, lines, NL, lo, hi, &fill, truth, alpha, 3,
                             0x3ffu, po, ao, co, it) == 0);
    CHECK(isfinite(co[0]) && co[0] < 1e-6);
    double steps[NPIX * 9], sg[NPIX * 9], H[NPIX * 81], He[NPIX * 81], hu[NPIX * 9];
    CHECK(oracle_population_steps(fg, ff, NPIX, POP, lo, hi, bp, steps) == 0);
    for (int i = 0; i < NPIX * 9; ++i)
        steps[i] = 0.01;
    CHECK(oracle_uncertainty(obs, sigma, mu, 1, lines, NL, lo, hi, truth, steps, 0x1ffu, sg, H,
                             He, hu) == 0);
    double q[3] = {0.3, -0.2, 0.5}, hq[3] = {0.1, 0.1, 0.1}, Hq[9], Hqe[9], sq[9];
    int32_t act[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    CHECK(oracle_sec6_hessian(quad, NULL, 3, q, hq, act, Hq, Hqe) == 0);
    CHECK(fabs(Hq[0] - 6.0) < 1e-8 && fabs(Hq[1] - 1.0) < 1e-8);
    double H9[81];
    memset(H9, 0, sizeof H9);
    for (int j = 0; j < 9; ++j)
        H9[j * 9 + j] = 2.0 + j;
    CHECK(oracle_sec6_sigmas(H9, act, 1.0, 9, sq) == 0);
    free(obs);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle under sanitizers: all checks passed\n");
    return 0;
}
