/*
 * FP64 CPU oracle for Milne-Eddington genetic-algorithm Stokes inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or constant generator with the HIP library.
 *
 * Method: Harker & Mighell, "A GPU-Computing Approach to Solar Stokes Profile
 * Inversion" (GENESIS).  Section references below are to that paper.
 *
 * Parameter vector of one model atmosphere (9 doubles, this order):
 *   0 B      field strength [G]
 *   1 incl   inclination psi to the line of sight [deg]
 *   2 azim   azimuth chi [deg]
 *   3 vlos   line-of-sight velocity [km/s], positive = redshift; it moves the
 *            line centre to lambda0 * (1 + vlos / c)   (stands in for the
 *            paper's free line-centre wavelength, Sec. 5 model vector)
 *   4 dopp   Doppler width Delta lambda_D [Angstrom]
 *   5 damp   damping parameter a
 *   6 eta0   line-to-continuum opacity ratio
 *   7 S0     source function at tau = 0
 *   8 S1     source function gradient (S1 = S0 * beta0 of Sec. 5)
 *
 * Parity of the genetic operators: the integer steps (Philox, tournament,
 * crossover, mutation) are pinned and compared bit-exactly.  The end-to-end
 * inversion is a stochastic heuristic whose general trajectory has no closed
 * form; it is pinned by the special cases that have one (without crossover
 * and mutation the loop only reselects generation 0, keeping its best; a
 * tournament over the whole population breeds copies of generation 0's
 * best), by determinism and resumption, and by recovered-parameter accuracy
 * on synthetic truth.
 */
#ifndef GENESIS_ORACLE_H
#define GENESIS_ORACLE_H

#include <stdint.h>

#define ORACLE_NPAR 9
#define ORACLE_MAXCOMP 64
#define ORACLE_MAXLINES 8
#define ORACLE_C_KMS 299792.458          /* speed of light [km/s] */

typedef struct {
    double lambda0;                    /* rest wavelength [Angstrom] */
    int32_t ncomp;                     /* Zeeman components */
    int32_t q[ORACLE_MAXCOMP];         /* M_lower - M_upper */
    double shift[ORACLE_MAXCOMP];      /* g_l M_l - g_u M_u, units of Delta lambda_B */
    double strength[ORACLE_MAXCOMP];   /* relative strength, each q group sums to 1 */
    double start;                      /* first wavelength sample [Angstrom] */
    double step;                       /* sample spacing [Angstrom] */
    int32_t nlam;                      /* samples for this line */
} oracle_line;

/* Faddeeva function w(x + i y) = exp(-z^2) erfc(-i z), y >= 0 (Sec. 5: Voigt
 * H = Re w and Faraday-Voigt L = Im w).  Valid for 0 <= y <= 1.5 to ~1e-14
 * absolute; returns NaN outside that strip. */
void oracle_faddeeva(double x, double y, double *re, double *im);

/* LS-coupling Lande factor of a term 2S+1 L_J; returns 0 for J = 0. */
double oracle_lande_ls(double S, double L, double J);
/* Wigner 3j symbol by the Racah sum (integer or half-integer arguments). */
double oracle_wigner3j(double j1, double j2, double j3, double m1, double m2, double m3);
/* Full Zeeman pattern of a J_l -> J_u dipole transition (Sec. 5: computed once
 * per inversion).  Writes up to cap components; returns the count or -1. */
int oracle_zeeman(double Jl, double gl, double Ju, double gu,
                  int32_t *q, double *shift, double *strength, int cap);

/* Stokes synthesis (Sec. 5, Unno-Rachkovsky solution).  par [n][9]; mu [n] or
 * NULL (= 1); out [n][4][L] with L = sum of nlam, lines concatenated. */
void oracle_me_synth(const double *par, int64_t n, const oracle_line *lines, int nlines,
                     const double *mu, double *out);

/* One model par with every component's Faddeeva value taken to first order
 * about its value at par0: w(z) ~ w(z0) + w'(z0)(z - z0), w' = -2 z w +
 * 2 i / sqrt(pi), z = v + i a of the component at par, z0 at par0; the rest
 * of the model (the propagation matrix and the Unno-Rachkovsky solution) is
 * evaluated at par.  par0 = par gives oracle_me_synth bit for bit.  This is
 * the model the refinement's Jacobian columns for B, v_los, the Doppler
 * width and the damping difference (oracle_lm.c).  out [4][L]. */
void oracle_me_synth_lin(const double *par0, const double *par, double mu,
                         const oracle_line *lines, int nlines, double *out);

/* Merit function (Sec. 5, chi-square equation) with w_i = 1/sigma_i:
 * chi2 = 1/nu sum_i sum_j (O - M)^2 / sigma_i^2, nu = 4L - 9.
 * par [npix][pop][9], obs [npix][4][L], sigma [npix][4], chi2 [npix][pop]. */
void oracle_chi2(const double *par, int64_t npix, int pop, const oracle_line *lines, int nlines,
                 const double *obs, const double *sigma, const double *mu, double *chi2);

/* Fill fraction (Sec. 5.2, see oracle_fill.c): the field-free profile of
 * each line as cubic polynomials in mu of its depth, width [A] and damping,
 * and the range of alpha. */
typedef struct {
    double depth[4], width[4], damp[4];
} oracle_fill_line;
typedef struct {
    double alpha_lo, alpha_hi;
    oracle_fill_line line[ORACLE_MAXLINES];
} oracle_fill;

/* N [nlam] of one line at mu for the model velocity vlos; 0, or -1 when the
 * width is not positive or the damping outside [0, 1.5] at this mu. */
int oracle_fill_profile(const oracle_line *ln, const oracle_fill_line *f, double mu, double vlos,
                        double *N);
/* alpha M(p) + (1 - alpha) I_c N e for n models (par [n][9], alpha [n],
 * mu [n] or NULL) -> out [n][4][L]; -1 (and NaN rows) where N is invalid. */
int oracle_me_synth_fill(const double *par, const double *alpha, int64_t n,
                         const oracle_line *lines, int nlines, const double *mu,
                         const oracle_fill *fill, double *out);
/* chi-square at the best alpha of each model and that alpha
 * (par [npix][pop][9] -> chi2, alpha [npix][pop]); nu = 4L - 10. */
void oracle_chi2_fill(const double *par, int64_t npix, int pop, const oracle_line *lines,
                      int nlines, const double *obs, const double *sigma, const double *mu,
                      const oracle_fill *fill, double *chi2, double *alpha);

/* Philox4x32-10 (Salmon et al. 2011). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Word n of the random stream (seed, pixel, generation, individual, purpose). */
uint32_t oracle_rng_word(uint64_t seed, uint32_t pixel, uint32_t gen, uint32_t indiv,
                         uint32_t purpose, uint32_t n);

/* Decoding operator E^-1 (Sec. 3, decode equation) for 16-bit genes. */
void oracle_decode(const uint16_t *genes, const double *lo, const double *hi, double *par);

/* Generation-0 population: genes [pop][9].  Individual i below n_seeded
 * encodes first guess i mod S of seed_par [S][9] (S = seed_sets, 0 reads as 1)
 * in the box [lo, hi] (exactly for i < S, jittered by up to +-jitter codes per
 * gene for the others); the rest are uniform random codes (or Sobol points).
 * seed_par, lo and hi may be NULL when n_seeded = 0. */
void oracle_ga_init(uint64_t seed, uint32_t pixel, int pop, int n_seeded, int jitter,
                    int seed_sets, const double *seed_par, const double *lo, const double *hi,
                    int init_mode, uint16_t *genes);

/* Sobol points (Sec. 5.6 initialisation and restarts): the first n primitive
 * polynomials over GF(2) (bit k = coefficient of x^k; returns how many were
 * found), the direction numbers V_k of the 9 dimensions, and point n. */
int oracle_sobol_polys(uint32_t *polys, int n);
void oracle_sobol_directions(uint32_t v[9][32]);
void oracle_sobol_point(uint32_t n, uint32_t out[9]);

/* Restart after generation t: genes_out = genes_in with the worst pop/2
 * replaced by Sobol points; replaced [pop] (may be NULL) flags them. */
void oracle_ga_restart(const uint16_t *genes_in, const double *fit, int pop, uint64_t seed,
                       uint32_t pixel, int t, int restart_every, uint16_t *genes_out,
                       int32_t *replaced);

/* One generation of the operators S, R, M of the standard GA (Sec. 3,
 * Algorithm 1) with elitism.  Produces generation `gen` (>= 1) from the
 * population genes_in [pop][9] and its fitness fit [pop].
 * Outputs: genes_out [pop][9]; parents [pop][2]; xpoint [pop] (0 = no
 * crossover); masks [pop][9] (mutation XOR masks); *elite.
 * Returns 0, or -1 on invalid arguments. */
int oracle_ga_step(const uint16_t *genes_in, const double *fit, int pop, int k,
                   double p_cross, double p_mut, uint64_t seed, uint32_t pixel, uint32_t gen,
                   uint16_t *genes_out, int32_t *parents, int32_t *xpoint, uint16_t *masks,
                   int32_t *elite);

/* Full inversion of npix pixels (Algorithm 1 run for G generations after the
 * initial evaluation).  Pixel p uses RNG pixel id pixel_base + p.
 * best_params [npix][9], best_chi2 [npix], status [npix] (0 ok, 1 non-finite
 * observation, 2 sigma <= 0 or non-finite, 3 invalid pixel box);
 * final_genes [npix][pop][9] and final_fit [npix][pop] may be NULL.
 * n_seeded > 0 seeds generation 0 of pixel p from seed_params
 * [npix][S][9] (S = seed_sets, 0 reads as 1) as oracle_ga_init does.  pixel_box [npix][2][9] (lo row, then hi row; may be
 * NULL) replaces [lo, hi] for each pixel: decoding, seeding and the result
 * use the pixel's box.  fill (may be NULL) makes the fitness the chi-square
 * at each individual's best fill fraction (oracle_fill.c); best_alpha [npix]
 * (needed then) receives the best individual's alpha, and a pixel whose
 * field-free profile is invalid at its mu gets status 4.  Returns 0 or -1. */
int oracle_ga_invert(const double *obs, const double *sigma, const double *mu, int64_t npix,
                     const oracle_line *lines, int nlines, const double *lo, const double *hi,
                     const double *pixel_box, const oracle_fill *fill, double *best_alpha,
                     int pop, int generations, int k, double p_cross, double p_mut,
                     uint64_t seed, uint32_t pixel_base, int n_seeded, int seed_jitter,
                     int seed_sets, const double *seed_params, int init_mode, int restart_every,
                     double *best_params, double *best_chi2, int32_t *status,
                     uint16_t *final_genes, double *final_fit);

/* Levenberg-Marquardt refinement in FP64 (see oracle_lm.c for the exact
 * steps): params_in [npix][9] -> params_out [npix][9], chi2_out [npix],
 * iters_done [npix] (may be NULL).  Pixels with non-finite observations or
 * sigma <= 0 give NaN.  Returns 0 or -1 (iterations < 0 or empty bounds). */
int oracle_lm_refine(const double *obs, const double *sigma, const double *mu, int64_t npix,
                     const oracle_line *lines, int nlines, const double *lo, const double *hi,
                     const double *params_in, int iterations, double *params_out,
                     double *chi2_out, int32_t *iters_done);

/* The same fit with only the parameters in free_mask (bit j = parameter j)
 * adjusted; the others keep their (clamped) starting values. */
int oracle_lm_fit(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const oracle_line *lines, int nlines, const double *lo, const double *hi,
                  const double *params_in, int iterations, uint32_t free_mask,
                  double *params_out, double *chi2_out, int32_t *iters_done);

/* The fit with the fill fraction of Sec. 5.2 as a tenth coordinate (see
 * oracle_lm.c): the model alpha M(p) + (1 - alpha) I_c N e of oracle_fill.c,
 * alpha in [fill->alpha_lo, fill->alpha_hi] from alpha_in [npix];
 * free_mask bits 0..8 the parameters, bit 9 alpha.  Outputs params_out
 * [npix][9], alpha_out [npix], chi2_out [npix] (nu = 4L - 10), iters_done
 * [npix] (may be NULL).  A pixel whose field-free profile is invalid at its
 * mu (or at its starting v_los) gives NaN like a bad observation. */
int oracle_lm_fit_fill(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const oracle_line *lines, int nlines, const double *lo, const double *hi,
                       const oracle_fill *fill, const double *params_in, const double *alpha_in,
                       int iterations, uint32_t free_mask, double *params_out,
                       double *alpha_out, double *chi2_out, int32_t *iters_done);

/* Sec. 6 uncertainties at p_opt [npix][9] (see oracle_unc.c): initial steps
 * steps [npix][9] (parameter units; e.g. oracle_population_steps), bounded
 * there as described; free_mask as for oracle_lm_fit.  Outputs sigma_out
 * [npix][9]; hess, hess_err [npix][9][9] (the symmetrised Hessian of the
 * merit function and the tableaux' error estimates) and steps_used [npix][9]
 * may be NULL.  Returns 0 or -1 (empty bounds, no free parameter). */
int oracle_uncertainty(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const oracle_line *lines, int nlines, const double *lo, const double *hi,
                       const double *p_opt, const double *steps, uint32_t free_mask,
                       double *sigma_out, double *hess, double *hess_err, double *steps_used);

/* Initial steps of Sec. 6 from a final population: genes [npix][pop][9],
 * fitness [npix][pop] -> steps [npix][9], the RMS deviation from p_opt over
 * the best max(2, pop/4) individuals (all of them if pop < 2). */
int oracle_population_steps(const uint16_t *genes, const double *fitness, int64_t npix, int pop,
                            const double *lo, const double *hi, const double *p_opt,
                            double *steps);

/* The same Hessian for any objective f of n <= 9 variables (for the pins),
 * and the variances from a Hessian: sigma_j^2 = [H^-1]_jj chi2 / M over the
 * active parameters (NaN inactive, +inf where H_jj = 0). */
int oracle_sec6_hessian(double (*f)(const double *, void *), void *ctx, int n, const double *p,
                        const double *h, const int32_t *active, double *hess, double *hess_err);
int oracle_sec6_sigmas(const double *hess, const int32_t *active, double chi2, int M,
                       double *out);

/* Threads the OpenMP loops would use. */
int oracle_num_threads(void);

#endif
