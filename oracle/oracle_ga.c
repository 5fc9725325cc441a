/*
 * FP64 oracle: the genetic algorithm of Sec. 3 (Algorithm 1) with 16-bit
 * genes stored one parameter per unsigned short (Sec. 4.2), driven by a
 * counter-based Philox4x32-10 random stream.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *  - random stream: word n of stream (seed, pixel, gen, indiv, purpose) is
 *    word n%4 of Philox4x32-10 with key (seed_lo, seed_hi) and counter
 *    (pixel, gen, indiv, purpose << 24 | n/4).  Purposes: 0 initial genes,
 *    1 tournaments, 2 crossover, 3 mutation.
 *  - selection S ("sampling without replacement", Sec. 3): tournament of k
 *    distinct contestants drawn with Floyd's algorithm; a uniform integer in
 *    [0, m] is (u32 * (m + 1)) >> 32; the winner has the lowest fitness, ties
 *    go to the lowest index, NaN counts as +infinity.
 *  - recombination R ("swap segments", Sec. 3): single-point crossover of the
 *    144-bit string (9 genes, bit 0 = most significant) with probability
 *    p_cross, point x in [1, 143].
 *  - mutation M (less-significant bits flip more often, Sec. 3): bit k of a
 *    gene (k = 0 MSB ... 15 LSB) flips with probability
 *    p_k = 2 p_mut (k + 1) / 17, realised as a 16-bit uniform below
 *    floor(p_k * 65536 + 0.5).
 *  - elitism: the best individual is copied unchanged into slot 0; slots
 *    1 .. pop-1 hold the children of pairs (2p+1, 2p+2).
 *  - seeding (Sec. 5.5: first guesses placed in the initial population):
 *    a pixel has S >= 1 first guesses (seed_sets); individual i of
 *    0 .. n_seeded-1 of generation 0 encodes guess i mod S,
 *    gene = floor(65535 clamp((p - u) / (v - u), 0, 1) + 0.5), the inverse of
 *    the decoding equation rounded to the nearest code; individuals i < S
 *    keep their guess exactly, individual i >= S adds to gene j the integer
 *    d - J, d uniform in [0, 2J] from word j of stream purpose 5
 *    (J = seed_jitter), clamped to [0, 65535]; a NaN first guess leaves that
 *    parameter's gene as drawn for an unseeded individual.
 *  - Sobol initialisation and restarts (Sec. 5.6): Sobol points (Bratley &
 *    Fox's construction) with dimension 0 the base-2 van der Corput sequence
 *    and dimension d >= 1 built on the d-th primitive polynomial over GF(2)
 *    (ordered by degree, then by value) with initial direction numbers all 1;
 *    each pixel XORs the 32-bit coordinates with a digital shift (word d of
 *    stream purpose 4, individual 0) and keeps the top 16 bits.  Generation
 *    0 takes points 0 .. pop-1.  A restart after generation t (t a multiple
 *    of restart_every, 0 < t < G) replaces the worst pop/2 individuals (the
 *    tournament order) by points pop + (t/restart_every - 1) (pop/2) + q,
 *    q = rank - (pop - pop/2), and re-evaluates them.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

double oracle__chi2_fill_single(const double *par, double mu, const oracle_line *lines,
                                int nlines, const double *obs, const double *sigma,
                                const oracle_fill *fill, double *scratch, double *alpha_out);
double oracle__chi2_single(const double *par, double mu, const oracle_line *lines, int nlines,
                           const double *obs, const double *sigma, double *scratch);
int oracle__total_samples(const oracle_line *lines, int nlines);

#define NGENE ORACLE_NPAR
#define GENE_BITS 16

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of the Philox S-box on a 4x32 counter with a
 * 2x32 key bumped by the Weyl constants between rounds. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        const uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t y0 = hi1 ^ x1 ^ k0;
        const uint32_t y1 = lo1;
        const uint32_t y2 = hi0 ^ x3 ^ k1;
        const uint32_t y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

uint32_t oracle_rng_word(uint64_t seed, uint32_t pixel, uint32_t gen, uint32_t indiv,
                         uint32_t purpose, uint32_t n)
{
    const uint32_t ctr[4] = {pixel, gen, indiv, (purpose << 24) | (n >> 2)};
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[n & 3u];
}

/* uniform integer in [0, m] */
static uint32_t uniform_upto(uint32_t word, uint32_t m)
{
    return (uint32_t)(((uint64_t)word * ((uint64_t)m + 1u)) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Decoding operator (Sec. 3, decode equation): with bit 0 the most
 * significant bit, the bit string of a gene is the unsigned value g, and
 * p = u + (v - u) g / (2^16 - 1). */
void oracle_decode(const uint16_t *genes, const double *lo, const double *hi, double *par)
{
    for (int j = 0; j < NGENE; ++j)
        par[j] = lo[j] + (hi[j] - lo[j]) * (double)genes[j] / 65535.0;
}

static int ranks_before(const double *fit, int a, int b);

/* ---- Sobol points ----------------------------------------------------- */

/* polynomial product modulo p (degree deg) over GF(2), operands reduced */
static uint32_t gf2_mulmod(uint32_t a, uint32_t b, uint32_t p, int deg)
{
    uint32_t r = 0;
    while (b) {
        if (b & 1u)
            r ^= a;
        b >>= 1;
        a <<= 1;
        if (a >> deg & 1u)
            a ^= p;
    }
    return r;
}

/* order of x modulo p: the smallest e >= 1 with x^e = 1 (0 if none up to 2^deg) */
static uint64_t gf2_order_of_x(uint32_t p, int deg)
{
    uint32_t x = deg == 1 ? (2u ^ p) : 2u, y = x;
    for (uint64_t e = 1; e <= (1ull << deg); ++e) {
        if (y == 1u)
            return e;
        y = gf2_mulmod(y, x, p, deg);
    }
    return 0;
}

int oracle_sobol_polys(uint32_t *polys, int n)
{
    int d = 0;
    for (int deg = 1; d < n && deg < 31; ++deg)
        for (uint32_t p = (1u << deg) | 1u; p < (2u << deg) && d < n; p += 2)
            if (gf2_order_of_x(p, deg) == (1ull << deg) - 1)
                polys[d++] = p;
    return d;
}

void oracle_sobol_directions(uint32_t v[NGENE][32])
{
    uint32_t polys[NGENE - 1];
    oracle_sobol_polys(polys, NGENE - 1);
    for (int k = 1; k <= 32; ++k)
        v[0][k - 1] = 1u << (32 - k);
    for (int d = 1; d < NGENE; ++d) {
        const uint32_t p = polys[d - 1];
        int s = 0;
        while (p >> (s + 1))
            ++s;
        uint32_t m[33];
        for (int k = 1; k <= 32; ++k) {
            if (k <= s) {
                m[k] = 1u;
            } else {
                uint32_t x = m[k - s] ^ (m[k - s] << s);
                for (int i = 1; i < s; ++i)
                    if (p >> (s - i) & 1u)
                        x ^= m[k - i] << i;
                m[k] = x;
            }
            v[d][k - 1] = m[k] << (32 - k);
        }
    }
}

void oracle_sobol_point(uint32_t n, uint32_t out[NGENE])
{
    uint32_t v[NGENE][32];
    oracle_sobol_directions(v);
    for (int d = 0; d < NGENE; ++d) {
        uint32_t x = 0;
        for (int k = 0; k < 32; ++k)
            if (n >> k & 1u)
                x ^= v[d][k];
        out[d] = x;
    }
}

static void sobol_genes(uint64_t seed, uint32_t pixel, uint32_t n, uint16_t *g)
{
    uint32_t x[NGENE];
    oracle_sobol_point(n, x);
    for (int d = 0; d < NGENE; ++d)
        g[d] = (uint16_t)((x[d] ^ oracle_rng_word(seed, pixel, 0u, 0u, 4u, (uint32_t)d)) >> 16);
}

/* Encoding: the gene whose decoded value lies nearest to p inside [u, v]. */
static uint16_t encode(double p, double lo, double hi)
{
    const double span = hi - lo;
    double u = (p - lo) / (span > 0.0 ? span : 1.0);
    if (u < 0.0)
        u = 0.0;
    if (u > 1.0)
        u = 1.0;
    return (uint16_t)floor(u * 65535.0 + 0.5);
}

void oracle_ga_init(uint64_t seed, uint32_t pixel, int pop, int n_seeded, int jitter,
                    int seed_sets, const double *seed_par, const double *lo, const double *hi,
                    int init_mode, uint16_t *genes)
{
    const int S = seed_sets < 1 ? 1 : seed_sets;
    for (int i = 0; i < pop; ++i) {
        uint16_t *g = genes + i * NGENE;
        if (init_mode == 1)
            sobol_genes(seed, pixel, (uint32_t)i, g);
        else
            for (int j = 0; j < NGENE; ++j)
                g[j] = (uint16_t)(oracle_rng_word(seed, pixel, 0u, (uint32_t)i, 0u, (uint32_t)j) >>
                                  16);
        if (!(i < n_seeded && seed_par))
            continue;
        const double *guess = seed_par + (i % S) * NGENE;
        for (int j = 0; j < NGENE; ++j) {
            if (isnan(guess[j]))
                continue;              /* no first guess for this parameter */
            int v = encode(guess[j], lo[j], hi[j]);
            if (i >= S) {
                const uint32_t w = oracle_rng_word(seed, pixel, 0u, (uint32_t)i, 5u, (uint32_t)j);
                v += (int)uniform_upto(w, 2u * (uint32_t)jitter) - jitter;
                v = v < 0 ? 0 : (v > 65535 ? 65535 : v);
            }
            g[j] = (uint16_t)v;
        }
    }
}

/* Restart after generation t: rank by fitness (tournament order), replace the
 * worst pop/2 by Sobol points; replaced[i] = 1 for those. */
void oracle_ga_restart(const uint16_t *genes_in, const double *fit, int pop, uint64_t seed,
                       uint32_t pixel, int t, int restart_every, uint16_t *genes_out,
                       int32_t *replaced)
{
    const int nrep = pop / 2;
    const uint32_t r = (uint32_t)(t / restart_every);
    for (int i = 0; i < pop; ++i) {
        int rank = 0;
        for (int j = 0; j < pop; ++j)
            rank += ranks_before(fit, j, i);
        const int q = rank - (pop - nrep);
        if (q >= 0)
            sobol_genes(seed, pixel, (uint32_t)pop + (r - 1u) * (uint32_t)nrep + (uint32_t)q,
                        genes_out + i * NGENE);
        else
            memcpy(genes_out + i * NGENE, genes_in + i * NGENE, sizeof(uint16_t) * NGENE);
        if (replaced)
            replaced[i] = q >= 0;
    }
}

/* fitness with NaN read as +infinity */
static double fit_key(double f)
{
    return isnan(f) ? INFINITY : f;
}

/* true if individual a ranks before individual b */
static int ranks_before(const double *fit, int a, int b)
{
    const double fa = fit_key(fit[a]), fb = fit_key(fit[b]);
    if (fa < fb)
        return 1;
    if (fa > fb)
        return 0;
    return a < b;
}

/* One tournament: k distinct contestants by Floyd's algorithm; returns the
 * winner. */
static int tournament(const double *fit, int pop, int k, uint64_t seed, uint32_t pixel,
                      uint32_t gen, uint32_t pair, int which)
{
    int chosen[64] = {0};
    int nchosen = 0;
    for (int i = 0; i < k; ++i) {
        const int j = pop - k + i;
        const uint32_t w = oracle_rng_word(seed, pixel, gen, pair, 1u, (uint32_t)(which * k + i));
        const int t = (int)uniform_upto(w, (uint32_t)j);
        int seen = 0;
        for (int c = 0; c < nchosen; ++c)
            if (chosen[c] == t)
                seen = 1;
        chosen[nchosen++] = seen ? j : t;
    }
    int best = chosen[0];
    for (int c = 1; c < nchosen; ++c)
        if (ranks_before(fit, chosen[c], best))
            best = chosen[c];
    return best;
}

/* mask of the bits of gene j that come from the first parent, for a cut
 * after bit position x of the 144-bit string */
static uint16_t first_parent_mask(int j, int x)
{
    const int lo = j * GENE_BITS;
    if (x >= lo + GENE_BITS)
        return 0xFFFFu;
    if (x <= lo)
        return 0x0000u;
    const int nfirst = x - lo; /* 1..15 most significant bits */
    return (uint16_t)(0xFFFFu << (GENE_BITS - nfirst));
}

int oracle_ga_step(const uint16_t *genes_in, const double *fit, int pop, int k,
                   double p_cross, double p_mut, uint64_t seed, uint32_t pixel, uint32_t gen,
                   uint16_t *genes_out, int32_t *parents, int32_t *xpoint, uint16_t *masks,
                   int32_t *elite)
{
    if (pop < 2 || k < 1 || k > pop || k > 64 || gen < 1 || !(p_cross >= 0.0 && p_cross <= 1.0) ||
        !(p_mut >= 0.0 && p_mut <= 1.0))
        return -1;

    /* integer thresholds of the two probabilistic operators */
    const double cross_thr = floor(p_cross * 4294967296.0);
    uint32_t mut_thr[GENE_BITS];
    for (int kbit = 0; kbit < GENE_BITS; ++kbit) {
        double t = floor(2.0 * p_mut * (double)(kbit + 1) / 17.0 * 65536.0 + 0.5);
        if (t > 65536.0)
            t = 65536.0;
        mut_thr[kbit] = (uint32_t)t;
    }

    /* elitism: best of the parent generation */
    int e = 0;
    for (int i = 1; i < pop; ++i)
        if (ranks_before(fit, i, e))
            e = i;
    *elite = e;
    memcpy(genes_out, genes_in + e * NGENE, sizeof(uint16_t) * NGENE);
    parents[0] = e;
    parents[1] = e;
    xpoint[0] = 0;
    memset(masks, 0, sizeof(uint16_t) * NGENE);

    for (int c = 1; c < pop; ++c) {
        const uint32_t pair = (uint32_t)((c - 1) / 2);
        const int second = (c - 1) % 2;
        /* selection */
        const int A = tournament(fit, pop, k, seed, pixel, gen, pair, 0);
        const int B = tournament(fit, pop, k, seed, pixel, gen, pair, 1);
        /* recombination */
        const uint32_t w0 = oracle_rng_word(seed, pixel, gen, pair, 2u, 0u);
        const uint32_t w1 = oracle_rng_word(seed, pixel, gen, pair, 2u, 1u);
        const int do_cross = (double)w0 < cross_thr;
        const int x = do_cross ? 1 + (int)uniform_upto(w1, NGENE * GENE_BITS - 2) : 0;
        const uint16_t *ga = genes_in + (second ? B : A) * NGENE;
        const uint16_t *gb = genes_in + (second ? A : B) * NGENE;
        uint16_t child[NGENE];
        for (int j = 0; j < NGENE; ++j) {
            const uint16_t m = do_cross ? first_parent_mask(j, x) : 0xFFFFu;
            child[j] = (uint16_t)((ga[j] & m) | (gb[j] & (uint16_t)~m));
        }
        /* mutation */
        uint16_t mask[NGENE];
        for (int j = 0; j < NGENE; ++j) {
            uint16_t mk = 0;
            for (int kbit = 0; kbit < GENE_BITS; ++kbit) {
                const uint32_t idx = (uint32_t)(j * GENE_BITS + kbit);
                const uint32_t w = oracle_rng_word(seed, pixel, gen, (uint32_t)c, 3u, idx / 2u);
                const uint32_t u16 = (idx & 1u) ? (w >> 16) : (w & 0xFFFFu);
                if (u16 < mut_thr[kbit])
                    mk |= (uint16_t)(1u << (GENE_BITS - 1 - kbit));
            }
            mask[j] = mk;
        }
        for (int j = 0; j < NGENE; ++j) {
            genes_out[c * NGENE + j] = (uint16_t)(child[j] ^ mask[j]);
            masks[c * NGENE + j] = mask[j];
        }
        parents[2 * c] = A;
        parents[2 * c + 1] = B;
        xpoint[c] = x;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Full inversion: Algorithm 1 with the evaluation operator F = chi-square of
 * the decoded model against the pixel's observation. */
int oracle_ga_invert(const double *obs, const double *sigma, const double *mu, int64_t npix,
                     const oracle_line *lines, int nlines, const double *lo_all,
                     const double *hi_all, const double *pixel_box, const oracle_fill *fill,
                     double *best_alpha, int pop, int generations, int k, double p_cross, double p_mut,
                     uint64_t seed, uint32_t pixel_base, int n_seeded, int seed_jitter,
                     int seed_sets, const double *seed_params, int init_mode, int restart_every,
                     double *best_params, double *best_chi2, int32_t *status,
                     uint16_t *final_genes, double *final_fit)
{
    if (pop < 2 || k < 1 || k > pop || k > 64 || generations < 0)
        return -1;
    if (n_seeded < 0 || n_seeded > pop || seed_jitter < 0 || (n_seeded > 0 && !seed_params) ||
        seed_sets < 0)
        return -1;
    if ((init_mode != 0 && init_mode != 1) || restart_every < 0)
        return -1;
    if (fill && (!best_alpha || nlines > ORACLE_MAXLINES ||
                 !(0.0 <= fill->alpha_lo && fill->alpha_lo <= fill->alpha_hi &&
                   fill->alpha_hi <= 1.0)))
        return -1;
    const int L = oracle__total_samples(lines, nlines);
    const int S = seed_sets < 1 ? 1 : seed_sets;
    int err = 0;
#pragma omp parallel
    {
        uint16_t *g0 = (uint16_t *)malloc(sizeof(uint16_t) * NGENE * (size_t)pop);
        uint16_t *g1 = (uint16_t *)malloc(sizeof(uint16_t) * NGENE * (size_t)pop);
        uint16_t *masks = (uint16_t *)malloc(sizeof(uint16_t) * NGENE * (size_t)pop);
        int32_t *par2 = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)pop);
        int32_t *xp = (int32_t *)malloc(sizeof(int32_t) * (size_t)pop);
        double *fit = (double *)malloc(sizeof(double) * (size_t)pop);
        double *scratch = (double *)malloc(sizeof(double) * 5 * (size_t)L);
        double *alph = (double *)malloc(sizeof(double) * (size_t)pop);
#pragma omp for schedule(dynamic, 1)
        for (int64_t p = 0; p < npix; ++p) {
            const double *o = obs + p * 4 * L;
            const double *s = sigma + p * 4;
            int st = 0;
            for (int i = 0; i < 4 * L; ++i)
                if (!isfinite(o[i]))
                    st = 1;
            for (int i = 0; i < 4; ++i)
                if (!(isfinite(s[i]) && s[i] > 0.0))
                    st = st ? st : 2;
            /* the pixel's own search box when given (Sec. 5.3 and 5.5 narrow
               it per pixel), else the common one */
            const double *lo = pixel_box ? pixel_box + p * 2 * NGENE : lo_all;
            const double *hi = pixel_box ? pixel_box + p * 2 * NGENE + NGENE : hi_all;
            if (pixel_box)
                for (int j = 0; j < NGENE; ++j)
                    if (!(isfinite(lo[j]) && isfinite(hi[j]) && hi[j] >= lo[j]))
                        st = st ? st : 3;
            const double m = mu ? mu[p] : 1.0;
            if (fill && !st)
                for (int l = 0; l < nlines; ++l)
                    if (oracle_fill_profile(&lines[l], &fill->line[l], m, 0.0, scratch) != 0)
                        st = 4;
            status[p] = st;
            if (st) {
                for (int j = 0; j < NGENE; ++j)
                    best_params[p * NGENE + j] = NAN;
                best_chi2[p] = NAN;
                if (fill)
                    best_alpha[p] = NAN;
                if (final_genes)
                    memset(final_genes + p * (int64_t)pop * NGENE, 0,
                           sizeof(uint16_t) * NGENE * (size_t)pop);
                if (final_fit)
                    for (int i = 0; i < pop; ++i)
                        final_fit[p * pop + i] = NAN;
                continue;
            }
            const uint32_t pix = pixel_base + (uint32_t)p;
            double par[NGENE];
            /* F of the decoded individual i (Sec. 5 chi-square, at its best
               fill fraction when fill is given) */
#define FITNESS(i)                                                                         \
    (fill ? oracle__chi2_fill_single(par, m, lines, nlines, o, s, fill, scratch, &alph[i]) \
          : oracle__chi2_single(par, m, lines, nlines, o, s, scratch))
            oracle_ga_init(seed, pix, pop, n_seeded, seed_jitter, S,
                           seed_params ? seed_params + p * S * NGENE : NULL, lo, hi, init_mode,
                           g0);
            for (int i = 0; i < pop; ++i) {
                oracle_decode(g0 + i * NGENE, lo, hi, par);
                fit[i] = FITNESS(i);
            }
            for (int t = 1; t <= generations; ++t) {
                if (restart_every > 0 && t - 1 > 0 && (t - 1) % restart_every == 0) {
                    /* restart of generation t - 1 (evaluated above), before breeding */
                    oracle_ga_restart(g0, fit, pop, seed, pix, t - 1, restart_every, g1, xp);
                    for (int i = 0; i < pop; ++i)
                        if (xp[i]) {
                            oracle_decode(g1 + i * NGENE, lo, hi, par);
                            fit[i] = FITNESS(i);
                        }
                    uint16_t *tmp = g0;
                    g0 = g1;
                    g1 = tmp;
                }
                int32_t e;
                if (oracle_ga_step(g0, fit, pop, k, p_cross, p_mut, seed, pix, (uint32_t)t, g1,
                                   par2, xp, masks, &e) != 0) {
#pragma omp atomic write
                    err = 1;
                    break;
                }
                uint16_t *tmp = g0;
                g0 = g1;
                g1 = tmp;
                for (int i = 0; i < pop; ++i) {
                    oracle_decode(g0 + i * NGENE, lo, hi, par);
                    fit[i] = FITNESS(i);
                }
            }
#undef FITNESS
            int b = 0;
            for (int i = 1; i < pop; ++i)
                if (ranks_before(fit, i, b))
                    b = i;
            oracle_decode(g0 + b * NGENE, lo, hi, best_params + p * NGENE);
            best_chi2[p] = fit[b];
            if (fill)
                best_alpha[p] = alph[b];
            if (final_genes)
                memcpy(final_genes + p * (int64_t)pop * NGENE, g0,
                       sizeof(uint16_t) * NGENE * (size_t)pop);
            if (final_fit)
                memcpy(final_fit + p * pop, fit, sizeof(double) * (size_t)pop);
        }
        free(g0);
        free(g1);
        free(alph);
        free(masks);
        free(par2);
        free(xp);
        free(fit);
        free(scratch);
    }
    return err ? -1 : 0;
}
