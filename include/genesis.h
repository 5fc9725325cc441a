/*
 * genesis.h -- C ABI of the MI355X (gfx950) library libgenesis_hip.so:
 * population-parallel genetic-algorithm inversion of solar Stokes profiles
 * under the Milne-Eddington model.
 *
 * Method: Harker & Mighell, "A GPU-Computing Approach to Solar Stokes Profile
 * Inversion" (GENESIS).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Array pointers are DEVICE memory owned by the caller unless stated.
 *    Struct pointers (lines, grids, bounds, config) are HOST memory, read
 *    during the call only.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *    asynchronous on that stream.  Apart from a serving session (gs_*),
 *    which owns the resident populations of its requests, the library
 *    allocates nothing on the device and keeps no device state between
 *    calls.
 *  - Return value: 0 on success or a negative ME_E* code; the message of the
 *    last failure on the calling thread is returned by me_last_error().  No
 *    C++ exception crosses this boundary.  On error nothing is launched.
 *  - Parameter vector of one Milne-Eddington atmosphere, GENESIS_NPAR = 9
 *    values in this order (Sec. 5 model vector; v_los stands in for the free
 *    line-centre wavelength and S1 = S0 beta0 for the source gradient):
 *      0 B [G]   1 inclination [deg]   2 azimuth [deg]   3 v_los [km/s]
 *      4 Doppler width [Angstrom]   5 damping a   6 eta0   7 S0   8 S1
 *  - Stokes arrays are [n][4][L] (I, Q, U, V), L = sum of grid[l].n over the
 *    lines, lines concatenated in the order given.  Observations are
 *    [npix][4][L]; noise is sigma [npix][4] with chi-square weights
 *    w_i = 1/sigma_i (Sec. 5 merit function, weights constant over
 *    wavelength).  mu (cosine of the heliocentric angle) is [npix] or NULL
 *    for mu = 1.
 *  - Genes are uint16 [.][9], one 16-bit gene per parameter (Sec. 4.2);
 *    bit 0 of the paper's bit string is the most significant bit.
 */
#ifndef GENESIS_H
#define GENESIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GENESIS_ABI_VERSION 5
#define GENESIS_NPAR 9
#define GENESIS_MAX_COMP 32   /* Zeeman components per line */
#define GENESIS_MAX_LINES 4
#define GENESIS_MAX_POP 1024
#define GENESIS_MAX_K 8       /* tournament size */

enum {
    ME_OK = 0,
    ME_EINVAL = -1, /* invalid argument (shape, range, NULL pointer) */
    ME_ENOMEM = -2, /* workspace too small / shared memory limit exceeded */
    ME_EHIP = -3,   /* a HIP runtime call failed */
    ME_EBUSY = -4   /* resource in use */
};

/* Zeeman pattern of one spectral line (Sec. 5: the full pattern of the
 * transition is computed once, at the start of an inversion).  Component c
 * has q[c] = M_lower - M_upper in {-1, 0, +1}, wavelength shift
 * shift[c] * Delta_lambda_B with shift = g_l M_l - g_u M_u and
 * Delta_lambda_B = 4.6686e-13 lambda0^2 B [Angstrom], and relative strength
 * strength[c]; strengths of each q group sum to 1. */
typedef struct {
    double lambda0_A;
    int32_t ncomp;
    int32_t q[GENESIS_MAX_COMP];
    double shift[GENESIS_MAX_COMP];
    double strength[GENESIS_MAX_COMP];
} me_line;

/* Wavelength samples of one line: lambda_j = start_A + j step_A, j < n. */
typedef struct {
    double start_A;
    double step_A;
    int32_t n;
} me_grid;

/* Search box u_j <= p_j <= v_j of the nine parameters (Sec. 3). */
typedef struct {
    double lo[GENESIS_NPAR];
    double hi[GENESIS_NPAR];
} me_bounds;

/* Genetic-algorithm configuration (Sec. 3, Algorithm 1).
 *  pop          population size, 2 .. GENESIS_MAX_POP
 *  generations  G >= 0 iterations after the initial evaluation
 *  tournament_k contestants per tournament, 1 .. min(pop, GENESIS_MAX_K)
 *  n_seeded     individuals 0 .. n_seeded-1 of generation 0 start from a
 *               first guess of the pixel instead of random genes (Sec. 5.5
 *               seeds the population with first guesses): individual i
 *               encodes guess i mod S of the pixel's S = seed_sets guesses,
 *               exactly for i < S; individual i >= S adds to each gene a
 *               uniform integer in [-seed_jitter, seed_jitter] (stream
 *               purpose 5), clamped to [0, 65535]; 0 = no seeding
 *  p_cross      probability of single-point crossover of a pair
 *  p_mut        mean per-bit mutation probability r; bit k (0 = MSB) flips
 *               with probability 2 r (k + 1) / 17
 *  seed         key of the counter-based random stream
 *  pixel_base   pixel p of the call draws random numbers as pixel
 *               pixel_base + p, so a map split into calls reproduces the
 *               single-call result
 *  seed_jitter  see n_seeded, 0 .. 32767
 *  seed_params  [npix][S][9] device array of first guesses (parameter
 *               units), used when n_seeded > 0; a NaN entry leaves that
 *               parameter's gene as drawn for an unseeded individual
 *  seed_sets    S, the first guesses per pixel in seed_params (0 reads as 1;
 *               at most GENESIS_MAX_POP); e.g. the four me_seeds guesses
 *  synth_precision  arithmetic of the profile synthesis inside ga_invert:
 *               GENESIS_SYNTH_NATIVE (that of the entry point) or
 *               GENESIS_SYNTH_FP16 (FP32 entry point only: Voigt and
 *               Faraday-Voigt profiles in packed FP16, two wavelengths per
 *               instruction, Unno-Rachkovsky and chi-square in FP32; needs a
 *               damping upper bound <= 1)
 *  init_mode    generation 0 (Sec. 5.6): 0 = uniform random genes (stream
 *               purpose 0); 1 = Sobol points 0 .. pop-1 (dimension 0 van der
 *               Corput, dimensions 1..8 from the first primitive polynomials
 *               over GF(2), initial direction numbers 1) XORed per pixel with
 *               a digital shift from stream purpose 4, top 16 bits per gene.
 *               Seeded slots (n_seeded) take precedence.
 *  restart_every  restarts (Sec. 5.6): 0 = none; R > 0 = after evaluating
 *               generation t with t % R == 0, 0 < t < G, the worst pop / 2
 *               individuals (NaN last, ties to the lower index) are replaced by
 *               Sobol points pop + (t/R - 1) (pop/2) + q (q = rank - (pop -
 *               pop/2)) of the pixel's shifted sequence and re-evaluated
 *  pixel_bounds [npix][2][9] device array (row 0 lo, row 1 hi, parameter
 *               units) or NULL: each pixel's own search box (Sec. 5.3 bounds
 *               the thermodynamic parameters per pixel from a pre-fit, Sec.
 *               5.5 restricts the inclination to one polarity), used by
 *               ga_init, ga_invert, ga_invert_f64 and the service for seeding,
 *               decoding and the result in place of the `bounds` argument
 *               (which must still be valid).  A pixel whose box is not finite
 *               with hi >= lo (or, for GENESIS_SYNTH_FP16, has damping
 *               outside [0, 1]) gets status 3 and NaN outputs.  ga_decode and
 *               ga_evaluate take the common box only.  See me_search_box. */
typedef struct {
    int32_t pop;
    int32_t generations;
    int32_t tournament_k;
    int32_t n_seeded;
    float p_cross;
    float p_mut;
    uint64_t seed;
    uint32_t pixel_base;
    int32_t seed_jitter;
    const float *seed_params;
    int32_t synth_precision;
    int32_t init_mode;
    int32_t restart_every;
    int32_t seed_sets;
    const float *pixel_bounds;
} ga_config;

#define GENESIS_SYNTH_NATIVE 0
#define GENESIS_SYNTH_FP16 1

/* Message of the last failure on this thread ("" if none). */
const char *me_last_error(void);
int genesis_abi_version(void);
/* sizeof of the argument structs as compiled into the library, for bindings
 * to check their own layouts against: which = 0 me_line, 1 me_grid,
 * 2 me_bounds, 3 ga_config, 4 me_fill; 0 for any other value. */
size_t genesis_struct_size(int32_t which);

/* ---- line data (host only, no device work) ------------------------------ */

/* Full Zeeman pattern of the dipole transition J_l -> J_u with Lande
 * factors g_l, g_u (Sec. 5; Table 1 lists the two Fe I lines).
 * Returns 0, or ME_EINVAL for |J_u - J_l| > 1, J_l = J_u = 0, half-integer
 * mismatch or more than GENESIS_MAX_COMP components. */
int me_line_from_terms(double lambda0_A, double Jl, double gl, double Ju, double gu,
                       me_line *out);
/* Effective triplet: three components at shifts -geff, 0, +geff. */
int me_line_triplet(double lambda0_A, double geff, me_line *out);

/* ---- forward model (Sec. 5) --------------------------------------------- */

/* Stokes synthesis: params [n][9] -> stokes [n][4][L] by the analytic
 * Unno-Rachkovsky solution I = S0 e + mu S1 (1 + eta0 Phi)^-1 e with the
 * Voigt and Faraday-Voigt profiles over every Zeeman component.
 * FP32: rational Voigt approximation (degree 6/7, max error 1.5e-7) in FP32
 * arithmetic.
 * n may be 0.  ME_EINVAL on NULL arrays (n > 0), nlines out of range, a grid
 * with n < 1, or an invalid line. */
int me_synth(const float *params, int64_t n, const me_line *lines, const me_grid *grids,
             int32_t nlines, const float *mu, float *stokes, void *stream);
/* FP32 parameters and Stokes vectors, profiles of the Zeeman components in
 * packed FP16 as in ga_config.synth_precision = GENESIS_SYNTH_FP16 (the same
 * device code); damping of every model must lie in [0, 1]. */
int me_synth_f16(const float *params, int64_t n, const me_line *lines, const me_grid *grids,
                 int32_t nlines, const float *mu, float *stokes, void *stream);
/* FP64 arithmetic with the Weideman N = 36 Faddeeva approximation. */
int me_synth_f64(const double *params, int64_t n, const me_line *lines, const me_grid *grids,
                 int32_t nlines, const double *mu, double *stokes, void *stream);

/* Merit function F (Sec. 5 chi-square): for pixel p and individual i,
 * chi2[p][i] = 1/nu sum_s sum_j ((obs[p][s][j] - M[s][j]) / sigma[p][s])^2,
 * nu = 4L - 9, M synthesised from params [npix][pop][9].  Accumulation:
 * per-Stokes sums of squared residuals over j ascending (FP32 in me_chi2,
 * FP64 in me_chi2_f64), then sum_s sum / sigma_s^2, then / nu.
 * Pixels with non-finite observations or sigma <= 0 give NaN. */
int me_chi2(const float *params, int64_t npix, int32_t pop, const float *obs, const float *sigma,
            const float *mu, const me_line *lines, const me_grid *grids, int32_t nlines,
            float *chi2, void *stream);
int me_chi2_f64(const double *params, int64_t npix, int32_t pop, const double *obs,
                const double *sigma, const double *mu, const me_line *lines,
                const me_grid *grids, int32_t nlines, double *chi2, void *stream);

/* ---- genetic operators (Sec. 3, Sec. 4.2) ------------------------------- */

/* Generation-0 population genes [npix][pop][9]: gene j of individual i of
 * pixel p = high 16 bits of word j of the random stream
 * (seed, pixel_base + p, generation 0, individual i, purpose 0), or the
 * seeded genes described at ga_config for i < n_seeded (bounds are needed
 * then, to encode the first guesses; otherwise they may be NULL). */
int ga_init(int64_t npix, const ga_config *cfg, const me_bounds *bounds, uint16_t *genes,
            void *stream);

/* Decoding operator E^-1 (Sec. 3 decode equation):
 * p_j = lo_j + (hi_j - lo_j) g_j / 65535, genes [n][9] -> params [n][9]. */
int ga_decode(const uint16_t *genes, int64_t n, const me_bounds *bounds, float *params,
              void *stream);

/* Evaluation F[E^-1(G)]: fitness [npix][pop] of genes [npix][pop][9]; the
 * same arithmetic as the fused loop of ga_invert. */
int ga_evaluate(const uint16_t *genes, int64_t npix, int32_t pop, const me_bounds *bounds,
                const float *obs, const float *sigma, const float *mu, const me_line *lines,
                const me_grid *grids, int32_t nlines, float *fitness, void *stream);
int ga_evaluate_f64(const uint16_t *genes, int64_t npix, int32_t pop, const me_bounds *bounds,
                    const double *obs, const double *sigma, const double *mu,
                    const me_line *lines, const me_grid *grids, int32_t nlines,
                    double *fitness, void *stream);

/* One generation of selection S, recombination R and mutation M with
 * elitism, producing generation `generation` (>= 1) of every pixel from
 * genes_in [npix][pop][9] and its fitness [npix][pop].
 *  - elite (best fitness, ties to the lowest index, NaN = +inf) -> slot 0;
 *  - slot c >= 1 is child (c-1)%2 of pair (c-1)/2: two tournaments of k
 *    distinct contestants (Floyd sampling), single-point crossover of the
 *    144-bit string with probability p_cross at a point in [1, 143], then a
 *    per-bit XOR mutation mask.
 * Outputs genes_out [npix][pop][9]; optional (NULL to skip): parents
 * [npix][pop][2], xpoint [npix][pop] (0 = no crossover), masks
 * [npix][pop][9], elite [npix].  genes_in and genes_out must not overlap. */
int ga_step(const uint16_t *genes_in, const float *fitness, int64_t npix, const ga_config *cfg,
            int32_t generation, uint16_t *genes_out, int32_t *parents, int32_t *xpoint,
            uint16_t *masks, int32_t *elite, void *stream);
int ga_step_f64(const uint16_t *genes_in, const double *fitness, int64_t npix,
                const ga_config *cfg, int32_t generation, uint16_t *genes_out, int32_t *parents,
                int32_t *xpoint, uint16_t *masks, int32_t *elite, void *stream);

/* ---- the whole inversion (Algorithm 1, device resident) ----------------- */

/* Restart of generation `generation` (a multiple of cfg->restart_every >= 1):
 * genes_out = genes_in with the worst pop / 2 individuals of every pixel
 * (by `fitness`, [npix][pop]) replaced as described for restart_every; the
 * caller then evaluates genes_out.  Sec. 5.6.  genes_in and genes_out must not
 * overlap. */
int ga_restart(const uint16_t *genes_in, const float *fitness, int64_t npix,
               const ga_config *cfg, int32_t generation, uint16_t *genes_out, void *stream);
int ga_restart_f64(const uint16_t *genes_in, const double *fitness, int64_t npix,
                   const ga_config *cfg, int32_t generation, uint16_t *genes_out, void *stream);

/* Device workspace ga_invert needs (bytes); currently 0: the population,
 * its fitness and the pixel's observation live in on-chip memory. */
size_t ga_workspace_bytes(int64_t npix, const ga_config *cfg);

/* Invert npix pixels: create P0, evaluate, then G times select, recombine,
 * mutate, decode and evaluate; one workgroup per pixel, one individual per
 * lane, a single launch.  Outputs best_params [npix][9] (decoded best
 * genotype of the last generation), best_chi2 [npix], status [npix]
 * (0 ok, 1 non-finite observation, 2 sigma <= 0 or non-finite, 3 invalid
 * pixel box (ga_config.pixel_bounds); outputs NaN for status != 0) -- status may be NULL; final_genes [npix][pop][9] and
 * final_fitness [npix][pop] may be NULL.  workspace/ws_bytes may be NULL/0.
 * When every workgroup fits on the device at once, the call first zeroes a
 * small per-device progress counter (a one-block kernel on `stream`) through
 * which the workgroups steer their waves' issue priority; calls that overlap
 * on one device share it, which changes the issue order only, never a
 * result. */
int ga_invert(const float *obs, const float *sigma, const float *mu, int64_t npix,
              const me_line *lines, const me_grid *grids, int32_t nlines,
              const me_bounds *bounds, const ga_config *cfg, float *best_params,
              float *best_chi2, int32_t *status, uint16_t *final_genes, float *final_fitness,
              void *workspace, size_t ws_bytes, void *stream);
int ga_invert_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const ga_config *cfg, double *best_params,
                  double *best_chi2, int32_t *status, uint16_t *final_genes,
                  double *final_fitness, void *workspace, size_t ws_bytes, void *stream);

/* ---- magnetic fill fraction (Sec. 5.2) ------------------------------------ */

/* A fraction alpha of the pixel is magnetic and the rest field-free: the
 * Stokes vector is alpha M(p) + (1 - alpha) I_c N(lambda) e, with M the
 * Milne-Eddington vector of the nine parameters, I_c = S0 + mu S1 its
 * continuum, e = (1, 0, 0, 0) and N the normalised field-free Stokes I
 * profile, a Voigt profile centred on the model's line centre:
 *   N = 1 - d(mu) H(v, a(mu)) / H(0, a(mu)),
 *   v = (lambda - lambda0 (1 + v_los / c)) / w(mu),
 * whose depth d, width w [A] and damping a are cubic polynomials in mu
 * (coefficients of mu^0 .. mu^3 per line; the paper fits them to measured
 * centre-to-limb variations it does not publish, so they are inputs).  A
 * pixel whose w(mu) <= 0 or a(mu) outside [0, 1.5] is invalid (status 4).
 * alpha is restricted to [alpha_lo, alpha_hi] within [0, 1]. */
typedef struct {
    double alpha_lo, alpha_hi;
    double depth[GENESIS_MAX_LINES][4];
    double width[GENESIS_MAX_LINES][4];
    double damp[GENESIS_MAX_LINES][4];
} me_fill;

/* Stokes vectors [n][4][L] of models params [n][9] with fill fractions
 * alpha [n] (mu [n] or NULL); NaN rows where the field-free profile is invalid. */
int me_synth_fill(const float *params, const float *alpha, int64_t n, const me_line *lines,
                  const me_grid *grids, int32_t nlines, const float *mu, const me_fill *fill,
                  float *stokes, void *stream);
int me_synth_fill_f64(const double *params, const double *alpha, int64_t n,
                      const me_line *lines, const me_grid *grids, int32_t nlines,
                      const double *mu, const me_fill *fill, double *stokes, void *stream);

/* ga_invert with the fill fraction as a tenth fitted parameter.  alpha enters
 * the model linearly, so every individual takes the alpha in [alpha_lo,
 * alpha_hi] that minimises its chi-square, in closed form, and its fitness is
 * that minimum (nu = 4L - 10); the genes, operators and outputs are those of
 * ga_invert, plus best_alpha [npix], the best individual's alpha.  Status 4
 * (NaN outputs) for a pixel whose field-free profile is invalid at its mu.
 * cfg->synth_precision = GENESIS_SYNTH_FP16 synthesises the magnetic
 * profiles in packed FP16 (the field-free profile, the mixture and the sums
 * in FP32); the FP64 entry point takes native synthesis only. */
int ga_invert_fill(const float *obs, const float *sigma, const float *mu, int64_t npix,
                   const me_line *lines, const me_grid *grids, int32_t nlines,
                   const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                   float *best_params, float *best_alpha, float *best_chi2, int32_t *status,
                   uint16_t *final_genes, float *final_fitness, void *stream);
int ga_invert_fill_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                       double *best_params, double *best_alpha, double *best_chi2,
                       int32_t *status, uint16_t *final_genes, double *final_fitness,
                       void *stream);

/* ---- FP64 refinement of a solution (non-linear least squares) ----------- */

/* Inverse-max weights of Sec. 5.4 as the sigma = 1 / w that the chi-square
 * calls take (sigma [npix][4], same precision as obs): for I the span of the
 * observed I of the pixel (largest minus smallest over every sample of every
 * line: continuum minus line core), for Q, U and V the largest |Q|, |U|,
 * |V|; each at least `floor` (finite, >= 0; a Stokes parameter without
 * signal, e.g. Q = U = V = 0 at zero field, would otherwise weigh
 * infinitely).  obs [npix][4][L] with L the grids' total samples; a pixel
 * with a non-finite sample gets four NaN (which ga_invert reports as status
 * 1).  Pass the result as the sigma of ga_invert, me_chi2 or me_refine_f64
 * to invert with this weighting instead of noise weights. */
int me_invmax_sigma(const float *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                    double floor, float *sigma, void *stream);
int me_invmax_sigma_f64(const double *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                        double floor, double *sigma, void *stream);

/* Heuristic first guesses [npix][9] (float) from the observed Stokes vectors
 * obs [npix][4][L] (FP64), for ga_config.seed_params: the paper seeds its
 * population with weak-field, centre-of-gravity and integral estimates
 * (Sec. 5.5).  Per line: v_los from the centre of gravity of the absorption
 * I_c - I; the longitudinal field from the centres of gravity of I + V and
 * I - V (their separation is 2 C gbar B cos(incl), C = 4.6686e-13 lambda0^2,
 * gbar the first moment of the red sigma group); the transverse field and
 * azimuth from the weak-field second-order relation of Q and U to the second
 * derivative of I (least squares); the Doppler width from the half-depth
 * width corrected for saturation; eta0 from the core depth with the source
 * function split mu S1 = 3/4 I_c, S0 = I_c / 4; damping the middle of its
 * range.  Lines combined by equivalent width; every value clamped into the
 * box.  mu [npix] may be NULL (mu = 1).  Every line needs >= 3 samples and a
 * red sigma group. */
int me_first_guess(const double *obs, const double *mu, int64_t npix, const me_line *lines,
                   const me_grid *grids, int32_t nlines, const me_bounds *bounds, float *params,
                   void *stream);

/* The four separate first guesses of Sec. 5.5, seeds [npix][4][9] (float,
 * parameter units; NaN = a parameter the seed leaves to the random draw),
 * for ga_config.seed_params with seed_sets = 4.  All four share the
 * thermodynamic estimates of me_first_guess (v_los, Doppler width, damping,
 * eta0, S0, S1); per line with I', I'' the sample differences (I' one-sided
 * at the window ends, I'' = 0 there), cg = C gbar, a = cg^2, summed over the
 * samples of every line:
 *   0 weak field (Auer et al.): least squares of V = -cg B_par I' and
 *     (Q, U) = -(1/4) a B_perp^2 (cos 2chi, sin 2chi) I'';
 *   1 integral relations (Ronan et al.): the same relations integrated,
 *     |B_par| = sum |V| / sum cg |I'| with the sign of -sum cg V I',
 *     B_perp^2 = 4 sum sqrt(Q^2 + U^2) / sum a |I''|, and the azimuth from the
 *     principal axis of the (Q, U) second moments, chi0 = atan2(2 sum QU,
 *     sum (Q^2 - U^2)) / 4 or chi0 + 90 deg, whichever has a projection
 *     Q cos 2chi + U sin 2chi <= 0 over the three samples around each line's
 *     minimum of I (where the pi component makes Q ~ -cos 2chi);
 *   2 centre of gravity (Rees & Semel): B = |B_par| of me_first_guess,
 *     inclination 0 or 180 by its sign, azimuth NaN;
 *   3 non-magnetic (full-disc runs): B = 0, both angles NaN.
 * Seeds 0 and 1 take B = hypot(B_par, B_perp), inclination atan2(B_perp,
 * B_par).  Each seed is made consistent with the pixel's box (pixel_bounds
 * [npix][2][9] as in ga_config, e.g. the polarity restriction, or the common
 * box when NULL): a non-finite B or thermodynamic value becomes the middle of
 * the box, the azimuth wraps into [0, 180), an inclination outside the box
 * becomes 180 minus itself, and every seeded value is clamped into the box.
 * Same requirements as me_first_guess. */
int me_seeds(const double *obs, const double *mu, int64_t npix, const me_line *lines,
             const me_grid *grids, int32_t nlines, const me_bounds *bounds,
             const float *pixel_bounds, float *seeds, void *stream);

/* Levenberg-Marquardt refinement in FP64 of one model per pixel, the local
 * least-squares polish of the genetic algorithm's best individual (the
 * machinery the paper uses for its non-magnetic pre-fit, Sec. 5.3, applied
 * here to the full model and the Sec. 5 chi-square).  In normalised
 * coordinates x_j = (p_j - lo_j)/(hi_j - lo_j), kept in [0, 1]: forward-
 * difference Jacobian (step 1e-7; for B, v_los, the Doppler width and the
 * damping the perturbed model takes each Zeeman component's Faddeeva value
 * to first order about the current one, w(z0 + dz) ~ w(z0) + w'(z0) dz with
 * w' = -2 z w + 2i/sqrt(pi)), normal equations, damped Cholesky steps
 * (lambda from 1e-3, /10 on success, x10 on failure, at most 10 trials per
 * iteration); stops after `iterations` or an iteration without progress.
 * params_in [npix][9] (need not lie inside the box: it is clamped);
 * outputs params_out [npix][9], chi2_out [npix] (FP64 model, same merit
 * function), iters_done [npix] (may be NULL).  Bounds need hi > lo for all
 * nine parameters.  Pixels with non-finite observations or sigma <= 0 give
 * NaN.  The uncertainties of Sec. 6 at the result: me_uncertainty_f64. */
int me_refine_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const double *params_in, int32_t iterations,
                  double *params_out, double *chi2_out, int32_t *iters_done, void *stream);

/* me_refine_f64 for the fill-fraction model of Sec. 5.2: alpha M(p) +
 * (1 - alpha) I_c N e (see me_fill), with alpha as a tenth coordinate
 * x_9 = (alpha - alpha_lo)/(alpha_hi - alpha_lo) fitted by the same steps;
 * nu = 4L - 10.  alpha_in [npix] starts it (e.g. ga_invert_fill's
 * best_alpha), alpha_out [npix] receives it; free_mask bits 0..8 are the
 * nine parameters, bit 9 alpha (0x3ff: all).  A pixel whose field-free
 * profile is invalid at its mu gives NaN like a bad observation.  Needs
 * alpha_hi > alpha_lo. */
int me_refine_fill_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const me_fill *fill, const double *params_in,
                       const double *alpha_in, int32_t iterations, uint32_t free_mask,
                       double *params_out, double *alpha_out, double *chi2_out,
                       int32_t *iters_done, void *stream);

/* Uncertainties of the fitted parameters (Sec. 6), FP64.  The Hessian H of
 * the merit function (the Sec. 5 chi-square, reduced by nu = 4L - 9) at
 * params_opt [npix][9] is the Jacobian of its gradient; both derivatives are
 * central differences extrapolated to zero step in a Neville tableau
 * (Ridders: steps h/1.4^k, k < 10, the entry of least estimated error, a
 * component stops once its diagonal moves by twice that error), the
 * gradient with one tableau per parameter, each Hessian column with one
 * tableau per gradient component on the gradients at p +- t e_j; H is then
 * symmetrised.  sigma_params [npix][9] = sqrt([H^-1]_jj chi2(p_opt) / M), M
 * the number of parameters in free_mask (bit j = parameter j; others held).
 * chi2(p_opt) takes the FP64 forward model (Weideman's Faddeeva expansion
 * with N = 36); the stencil points of the derivatives take N = 28 (error
 * about 2e-12, smooth in z, far below what the differences resolve).
 * steps [npix][9] are the initial steps in parameter units (Sec. 6 takes
 * them from the spread of the final population: ga_population_steps); each
 * is bounded to [1e-4, 0.1] (hi - lo) and to half the distance to the
 * nearer bound, and a parameter within 1e-4 (hi - lo) of a bound is held.
 * Per parameter: NaN if held, +infinity if H_jj = 0 (the merit function does
 * not depend on it; left out of the inverse), NaN for all when the rest of H
 * is not positive definite; NaN for pixels with non-finite observations or
 * parameters or sigma <= 0.  Optional outputs (may be NULL): hessian and
 * hessian_err [npix][9][9] (H and the tableaux' error estimates; 0 in the
 * rows and columns of held parameters), steps_used [npix][9].  About 1e4
 * merit-function evaluations per pixel (once per pixel, after the search). */
int me_uncertainty_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const double *params_opt, const double *steps,
                       uint32_t free_mask, double *sigma_params, double *hessian,
                       double *hessian_err, double *steps_used, void *stream);

/* Initial steps of Sec. 6 from a final population (ga_invert's final_genes
 * [npix][pop][9] and final_fitness [npix][pop]): steps [npix][9] = the
 * root-mean-square deviation from params_opt [npix][9] of each parameter
 * over the best max(2, pop/4) individuals (fitness order, NaN last, ties to
 * the lower index; every individual if pop < 2), decoded in `bounds`. */
int ga_population_steps(const uint16_t *genes, const float *fitness, int64_t npix, int32_t pop,
                        const me_bounds *bounds, const double *params_opt, double *steps,
                        void *stream);
int ga_population_steps_f64(const uint16_t *genes, const double *fitness, int64_t npix,
                            int32_t pop, const me_bounds *bounds, const double *params_opt,
                            double *steps, void *stream);

/* Non-magnetic pre-fit (Sec. 5.3): before the genetic search the paper fits
 * a non-magnetic model to the observed Stokes I by Levenberg-Marquardt and
 * uses the thermodynamic values only to confine the search.  This is the
 * me_refine_f64 iteration (same coordinates, steps and stopping rule) with B
 * held at 0, so neither field angle enters the model and Q = U = V = 0,
 * adjusting v_los, the Doppler width, damping, eta0, S0 and S1 from
 * params_in [npix][9] (its B is ignored; e.g. me_first_guess output).  The
 * box must contain B = 0 (ME_EINVAL otherwise).  Outputs params_out [npix][9]
 * (B = 0), chi2_out [npix] (the full four-Stokes merit function, whose Q, U,
 * V terms do not depend on the fitted parameters), iters_done [npix] (may be
 * NULL); NaN for pixels with non-finite observations or sigma <= 0. */
int me_prefit_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const double *params_in, int32_t iterations,
                  double *params_out, double *chi2_out, int32_t *iters_done, void *stream);

/* Per-pixel search boxes box [npix][2][9] (float; row 0 lo, row 1 hi) for
 * ga_config.pixel_bounds, starting from `bounds`:
 *  - with prefit [npix][9] (me_prefit_f64 output; may be NULL), the ranges of
 *    Sec. 5.3: a non-magnetic fit absorbs Zeeman broadening, so the Doppler
 *    width is bounded above by 1.1 x its pre-fit value and the damping by
 *    1.5 x its pre-fit value + 0.1 (hi - lo); eta0 is confined to [f/8, 8 f]
 *    and S1 (the paper's beta0) to [f/1.5, 1.5 f] about the pre-fit value f
 *    (all clipped to `bounds`; a non-finite or non-positive f leaves the
 *    range as it was);
 *  - with polarity_nsigma > 0, the polarity restriction of Sec. 5.5: with
 *    x_j the sample offsets from each line's centre of gravity of I_c - I
 *    (I_c the pixel's largest I), the first moment s = sum_lines sum_j x_j
 *    V_j is negative for inclinations below 90 degrees; when |s| exceeds
 *    polarity_nsigma x sigma_V x sqrt(sum x_j^2) the inclination range
 *    becomes its intersection with [0, 90] (s < 0) or [90, 180] (s > 0),
 *    unless that intersection is empty.  polarity_nsigma <= 0 skips it (obs
 *    and sigma may then be NULL).
 * obs [npix][4][L] and sigma [npix][4] FP64, as for me_first_guess. */
int me_search_box(const double *obs, const double *sigma, int64_t npix, const me_line *lines,
                  const me_grid *grids, int32_t nlines, const me_bounds *bounds,
                  const double *prefit, double polarity_nsigma, float *box, void *stream);

/* ---- learned proposal (first guesses for seeding) ---------------------- */

/* A multilayer perceptron maps a pixel's Stokes vector to a first guess of
 * its parameters, which seeds part of generation 0 (ga_config.n_seeded); the
 * paper seeds its population with heuristic first guesses (Sec. 5.5) and
 * cites neural-network inversion (Sec. 1).  Fixed architecture: 1024 inputs
 * (4 Stokes x 256 samples divided by the pixel's maximum of I) -> three GELU
 * layers of 512 -> 9 outputs, the parameters scaled to [0, 1] by the search
 * box (the azimuth periodic with period 1).  Parameters: one FP32 array of
 * mlp_param_count() values, layer by layer W[out][in] then b[out].  Matrix
 * products: BF16 operands with FP32 accumulation on the matrix cores
 * (precision 0) or FP32 on the vector units (precision 1, for checks). */
int64_t mlp_param_count(void);
/* Device workspace for a batch (activations and a BF16 weight copy). */
size_t mlp_workspace_bytes(int64_t batch);
/* He-normal weights, zero biases, from the counter-based stream. */
int mlp_init(float *master, uint64_t seed, void *stream);
/* x [npix][1024] = obs [npix][4][L] / max_j I_j, L = 256 required. */
int mlp_features(const float *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                 float *x, void *stream);
/* y [n][9] = network(x [n][1024]). */
int mlp_forward(const float *master, const float *x, int64_t n, int32_t precision, float *y,
                void *workspace, size_t ws_bytes, void *stream);
/* mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, with the workspace in a file-scope device array of the
 * library (about 20 MiB per device, held until the process ends) instead of
 * a workspace argument; it allocates nothing.  n must lie in [1,
 * mlp_noalloc_max_rows()] (ME_EINVAL otherwise: split larger batches).  The
 * caller still owns master, x [n][1024] and y [n][9] (device).  Every call
 * on one device shares that device's array: calls that overlap on one
 * device (different streams, or threads) race and must be serialised by the
 * caller. */
int64_t mlp_noalloc_max_rows(void);
int mlp_forward_noalloc(const float *master, const float *x, int64_t n, int32_t precision,
                        float *y, void *stream);
/* Gradient of loss = mean_b sum_j d_bj^2, d = y - target (azimuth d taken
 * modulo 1), into grad [param_count]; *loss (device) receives the loss. */
int mlp_grad(const float *master, const float *x, const float *target, int64_t batch,
             int32_t precision, float *grad, float *loss, void *workspace, size_t ws_bytes,
             void *stream);
/* One Adam step (beta 0.9, 0.999, eps 1e-8, bias-corrected; step >= 1). */
int mlp_adam(float *master, float *m, float *v, const float *grad, int32_t step, float lr,
             void *stream);
/* Training examples n, counter-indexed from `first`: parameters [n][9]
 * uniform in the box (v_los normal about the centre, sigma = width / 10,
 * clipped) and their scaled targets [n][9]. */
int mlp_draw_examples(uint64_t seed, int64_t first, int64_t n, const me_bounds *bounds,
                      float *params, float *target, void *stream);
/* stokes [n][4][L] += N(0, (sigma_rel (S0 + S1))^2), mu = 1. */
int mlp_add_noise(uint64_t seed, int64_t first, const float *params, int64_t n,
                  const me_grid *grids, int32_t nlines, float sigma_rel, float *stokes,
                  void *stream);
/* params [n][9] = box position of network outputs y [n][9] (clamped). */
int mlp_unscale(const float *y, int64_t n, const me_bounds *bounds, float *params, void *stream);
/* Device workspace of mlp_train for a batch. */
size_t mlp_train_workspace_bytes(int64_t batch);
/* `steps` Adam steps on fresh synthetic examples, all on `stream`: step
 * t = first_step + s draws examples (t - 1) batch ... t batch - 1 of stream
 * `seed` (mlp_draw_examples), synthesises them with me_synth (mu = 1), adds
 * noise (mlp_add_noise), normalises (mlp_features), computes the gradient
 * (mlp_grad) and applies mlp_adam with step number t.  losses [steps]
 * (device) receives each step's loss.  m and v start at zero for
 * first_step = 1 and carry over between calls. */
int mlp_train(float *master, float *m, float *v, int32_t first_step, int32_t steps,
              int64_t batch, float lr, uint64_t seed, const me_line *lines, const me_grid *grids,
              int32_t nlines, const me_bounds *bounds, float sigma_rel, int32_t precision,
              float *losses, void *workspace, size_t ws_bytes, void *stream);

/* ---- continuous-batching service -------------------------------------- */

/* A session inverts a stream of requests (tiles of pixels), the near real-time
 * use the paper aims at (Sec. 7).  gs_submit queues a request: the same
 * arguments as ga_invert (device arrays owned by the caller, which must stay
 * valid until the request is done; outputs are written when it finishes).
 * Each gs_step admits queued requests in arrival order while their resident
 * populations (npix x pop x (9 x 2 + 4) bytes, 256-byte aligned) fit in the
 * session's budget, then advances every resident request by up to
 * gens_per_step generations in one launch on `stream` (the first step of a
 * request also creates and evaluates its generation 0); finished requests
 * release their memory at once.  A request's result is bit-identical to
 * ga_invert with the same arguments, whatever else is resident.
 * gs_poll sets *done to 1 when the request's outputs are complete on the
 * device, 0 while queued or running, -1 if cancelled.  gs_cancel drops a
 * queued request at once and a resident one at the next step.  All calls
 * on one session are serialised by a lock; calls of different sessions on
 * one device may overlap.  gs_submit returns ME_ENOMEM for a request larger
 * than the whole budget.  The budget counts only what the session owns (the
 * resident populations), not the caller's input and output arrays.
 * Each gs_step waits on the device for the session's previous step, on
 * whatever stream that one ran, so steps may come on different streams.
 * cfg->synth_precision may select FP16 profile synthesis (damping bounds
 * within [0, 1], as for ga_invert); gs_submit_fill serves the fill-fraction
 * merit.  Requests of every kind share each launch. */
int gs_create(size_t hbm_budget_bytes, int32_t gens_per_step, void **session);
int gs_submit(void *session, const float *obs, const float *sigma, const float *mu, int64_t npix,
              const me_line *lines, const me_grid *grids, int32_t nlines,
              const me_bounds *bounds, const ga_config *cfg, float *best_params,
              float *best_chi2, int32_t *status, uint64_t *request_id);
/* gs_submit for the fill-fraction merit of Sec. 5.2 (as ga_invert_fill):
 * every individual takes its best alpha in [fill->alpha_lo, fill->alpha_hi]
 * in closed form; best_alpha [npix] (device, caller-owned) receives the best
 * individual's alpha; FP16 synthesis as in ga_invert_fill.  A
 * served tile equals ga_invert_fill of it bit for bit. */
int gs_submit_fill(void *session, const float *obs, const float *sigma, const float *mu,
                   int64_t npix, const me_line *lines, const me_grid *grids, int32_t nlines,
                   const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                   float *best_params, float *best_alpha, float *best_chi2, int32_t *status,
                   uint64_t *request_id);
int gs_step(void *session, void *stream);
/* Admission by compute as well as memory: with max_pixels > 0 a queued request
 * is admitted only while the resident pixels (plus its own) stay within
 * max_pixels, or when nothing is resident.  Every resident request shares each
 * launch, so admitting everything the memory budget allows makes all of them
 * finish late when the device is already full; a cap near the pixels that
 * fill the device (one workgroup each, about 2048 on 256 compute units) keeps
 * completions close to arrival order while small tiles still share launches.
 * 0 (the default) removes the cap.  Takes effect at the next gs_step. */
int gs_set_max_resident_pixels(void *session, int64_t max_pixels);
int gs_poll(void *session, uint64_t request_id, int32_t *done);
int gs_cancel(void *session, uint64_t request_id);
/* Forget a request whose outputs are complete (gs_poll gave 1) or that was
 * cancelled (-1): the session drops its record, after which its id is
 * unknown; the caller may then reuse or free the request's arrays.  A
 * long-running session must release what it has collected, or its records
 * grow without bound.  ME_EBUSY while the request is queued, resident or
 * still running on the device. */
int gs_release(void *session, uint64_t request_id);
int gs_stats(void *session, int64_t *queued, int64_t *resident, size_t *bytes_in_use);
/* Number of requests the session still holds records of (queued, resident,
 * and finished or cancelled but not yet released). */
int gs_tracked(void *session, int64_t *n);
int gs_destroy(void *session);

#ifdef __cplusplus
}
#endif

#endif /* GENESIS_H */
