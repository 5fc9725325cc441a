/*
 * FP64 oracle: Zeeman pattern, Faddeeva function, Milne-Eddington Stokes
 * synthesis and the chi-square merit function.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain definitions, no blocking,
 * no fusion, no approximation beyond the stated truncation of the Faddeeva sum.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_ZEEMAN_K 4.6686e-13       /* e / (4 pi m_e c^2) [1/(Angstrom G)] */

/* ------------------------------------------------------------------------ */
/* Faddeeva function.
 *
 * Sec. 5 builds the propagation matrix from the Voigt and Faraday-Voigt
 * profiles; we take H(a,v) = Re w(v + i a) and L(a,v) = Im w(v + i a) with
 * w(z) = exp(-z^2) erfc(-i z).
 *
 * Evaluation: w(z) = exp(-z^2) + (2 i / sqrt(pi)) F(z), where F is Dawson's
 * integral, and F is computed from Rybicki's sampling-theorem series
 *   F(z) = lim_{h->0} (1/sqrt(pi)) sum_{n odd} exp(-(z - n h)^2) / n,
 * (G. B. Rybicki, Computers in Physics 3, 85, 1989).  With h = 0.2 the
 * aliasing error is of order exp(-(pi/(2h))^2 + pi y / h), below 1e-14 for
 * y <= 1.5; terms with |x - n h| > 7 are below 1e-21 and dropped. */
void oracle_faddeeva(double x, double y, double *re, double *im)
{
    if (!(y >= 0.0 && y <= 1.5) || !(fabs(x) <= 1.0e5)) {
        *re = NAN;
        *im = NAN;
        return;
    }
    const double h = 0.2, R = 7.0;
    const double complex z = x + I * y;
    double complex sum = 0.0;
    const long nlo = (long)floor((x - R) / h) - 1;
    const long nhi = (long)ceil((x + R) / h) + 1;
    for (long n = nlo; n <= nhi; ++n) {
        if ((n & 1L) == 0)
            continue;
        const double complex d = z - (double)n * h;
        sum += cexp(-d * d) / (double)n;
    }
    const double complex w = cexp(-z * z) + (2.0 * I / M_PI) * sum;
    *re = creal(w);
    *im = cimag(w);
}

/* ------------------------------------------------------------------------ */
/* Zeeman pattern (Sec. 5: the full pattern of the transition is computed once
 * at the start of an inversion; Table 1 gives the terms of the two lines). */

double oracle_lande_ls(double S, double L, double J)
{
    if (J == 0.0)
        return 0.0;
    return 1.0 + (J * (J + 1.0) + S * (S + 1.0) - L * (L + 1.0)) / (2.0 * J * (J + 1.0));
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i)
        f *= (double)i;
    return f;
}

/* True when 2*x is an integer (within rounding of the inputs). */
static int twice_int(double x, int *out)
{
    const double t = 2.0 * x;
    const double r = floor(t + 0.5);
    if (fabs(t - r) > 1e-9)
        return 0;
    *out = (int)r;
    return 1;
}

/* Racah's closed formula for the 3j symbol. */
double oracle_wigner3j(double j1, double j2, double j3, double m1, double m2, double m3)
{
    int J1, J2, J3, M1, M2, M3; /* doubled values */
    if (!twice_int(j1, &J1) || !twice_int(j2, &J2) || !twice_int(j3, &J3) ||
        !twice_int(m1, &M1) || !twice_int(m2, &M2) || !twice_int(m3, &M3))
        return 0.0;
    if (M1 + M2 + M3 != 0)
        return 0.0;
    if (abs(M1) > J1 || abs(M2) > J2 || abs(M3) > J3)
        return 0.0;
    if (((J1 + M1) & 1) || ((J2 + M2) & 1) || ((J3 + M3) & 1))
        return 0.0;
    if (J3 < abs(J1 - J2) || J3 > J1 + J2 || ((J1 + J2 + J3) & 1))
        return 0.0;
    /* undoubled integer combinations */
    const int a = (J1 + J2 - J3) / 2, b = (J1 - J2 + J3) / 2, c = (-J1 + J2 + J3) / 2;
    const int d = (J1 + J2 + J3) / 2 + 1;
    const double tri = factorial(a) * factorial(b) * factorial(c) / factorial(d);
    const double pre = factorial((J1 + M1) / 2) * factorial((J1 - M1) / 2) *
                       factorial((J2 + M2) / 2) * factorial((J2 - M2) / 2) *
                       factorial((J3 + M3) / 2) * factorial((J3 - M3) / 2);
    double sum = 0.0;
    for (int k = 0; k <= 200; ++k) {
        const int t1 = (J3 - J2 + M1) / 2 + k;
        const int t2 = (J3 - J1 - M2) / 2 + k;
        const int t3 = (J1 + J2 - J3) / 2 - k;
        const int t4 = (J1 - M1) / 2 - k;
        const int t5 = (J2 + M2) / 2 - k;
        if (t3 < 0 || t4 < 0 || t5 < 0)
            break;
        if (t1 < 0 || t2 < 0)
            continue;
        const double den = factorial(k) * factorial(t1) * factorial(t2) * factorial(t3) *
                           factorial(t4) * factorial(t5);
        sum += ((k & 1) ? -1.0 : 1.0) / den;
    }
    const int ph = (J1 - J2 - M3) / 2;
    const double sign = (ph & 1) ? -1.0 : 1.0;
    return sign * sqrt(tri) * sqrt(pre) * sum;
}

int oracle_zeeman(double Jl, double gl, double Ju, double gu,
                  int32_t *q, double *shift, double *strength, int cap)
{
    int TJl, TJu;
    if (!twice_int(Jl, &TJl) || !twice_int(Ju, &TJu) || TJl < 0 || TJu < 0)
        return -1;
    if (abs(TJl - TJu) > 2 || (TJl == 0 && TJu == 0))
        return -1;
    int n = 0;
    for (int TMu = -TJu; TMu <= TJu; TMu += 2) {
        for (int TMl = -TJl; TMl <= TJl; TMl += 2) {
            const int Tq = TMl - TMu;
            if (Tq < -2 || Tq > 2)
                continue;
            const double Mu = 0.5 * TMu, Ml = 0.5 * TMl, qq = 0.5 * Tq;
            const double t = oracle_wigner3j(Ju, Jl, 1.0, -Mu, Ml, -qq);
            const double s = 3.0 * t * t;
            if (s <= 1e-14)
                continue;
            if (n >= cap)
                return -1;
            q[n] = Tq / 2;
            shift[n] = gl * Ml - gu * Mu;
            strength[n] = s;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Milne-Eddington synthesis (Sec. 5).
 *
 * K = 1 + eta0 Phi with the absorption (eta) and magneto-optical (rho)
 * elements built from the three Zeeman groups b (q = -1), p (q = 0) and
 * r (q = +1); the source function S0 + S1 tau gives the emergent vector
 * I = S0 e + mu S1 K^-1 e, which equals the paper's
 * Ic [(1 - beta) 1 + beta K^-1] e with Ic = S0 + mu S1 and
 * beta = mu beta0 / (1 + mu beta0), beta0 = S1/S0, written so that S0 = 0
 * is allowed.  K^-1 e is obtained by solving K x = e with Gaussian
 * elimination (partial pivoting). */

static void solve4(double A[4][4], double b[4], double x[4])
{
    int perm[4] = {0, 1, 2, 3};
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (fabs(A[perm[r]][col]) > fabs(A[perm[piv]][col]))
                piv = r;
        const int t = perm[col];
        perm[col] = perm[piv];
        perm[piv] = t;
        const int pr = perm[col];
        for (int r = col + 1; r < 4; ++r) {
            const int rr = perm[r];
            const double f = A[rr][col] / A[pr][col];
            for (int c = col; c < 4; ++c)
                A[rr][c] -= f * A[pr][c];
            b[rr] -= f * b[pr];
        }
    }
    for (int col = 3; col >= 0; --col) {
        const int pr = perm[col];
        double s = b[pr];
        for (int c = col + 1; c < 4; ++c)
            s -= A[pr][c] * x[c];
        x[col] = s / A[pr][col];
    }
}

static int total_samples(const oracle_line *lines, int nlines)
{
    int L = 0;
    for (int l = 0; l < nlines; ++l)
        L += lines[l].nlam;
    return L;
}

/* Stokes vector at one sample from the group profiles phi (absorption) and
 * psi (dispersion) of the blue, pi and red components (Sec. 5): the
 * propagation matrix and the Unno-Rachkovsky solution for the model par. */
static void stokes_from_profiles(const double *par, double mu, const double phi[3],
                                 const double psi[3], double st[4])
{
    const double gam = par[1] * M_PI / 180.0;
    const double chi = par[2] * M_PI / 180.0;
    const double eta0 = par[6];
    const double S0 = par[7];
    const double S1 = par[8];
    const double sg = sin(gam), cg = cos(gam);
    const double c2x = cos(2.0 * chi), s2x = sin(2.0 * chi);
    const double pb = phi[0], pp = phi[1], pr = phi[2];
    const double qb = psi[0], qp = psi[1], qr = psi[2];
    const double etaI = 0.5 * eta0 * (pp * sg * sg + 0.5 * (pb + pr) * (1.0 + cg * cg));
    const double etaQ = 0.5 * eta0 * (pp - 0.5 * (pb + pr)) * sg * sg * c2x;
    const double etaU = 0.5 * eta0 * (pp - 0.5 * (pb + pr)) * sg * sg * s2x;
    const double etaV = 0.5 * eta0 * (pr - pb) * cg;
    const double rhoQ = 0.5 * eta0 * (qp - 0.5 * (qb + qr)) * sg * sg * c2x;
    const double rhoU = 0.5 * eta0 * (qp - 0.5 * (qb + qr)) * sg * sg * s2x;
    const double rhoV = 0.5 * eta0 * (qr - qb) * cg;
    double K[4][4] = {
        {1.0 + etaI, etaQ, etaU, etaV},
        {etaQ, 1.0 + etaI, rhoV, -rhoU},
        {etaU, -rhoV, 1.0 + etaI, rhoQ},
        {etaV, rhoU, -rhoQ, 1.0 + etaI},
    };
    double e[4] = {1.0, 0.0, 0.0, 0.0}, x[4];
    solve4(K, e, x);
    st[0] = S0 + mu * S1 * x[0];
    st[1] = mu * S1 * x[1];
    st[2] = mu * S1 * x[2];
    st[3] = mu * S1 * x[3];
}

/* Reduced wavelength of component c of a line at sample lam for the model
 * par (Sec. 5: line centre shifted by v_los, Zeeman shift in units of the
 * Doppler width). */
static double component_v(const double *par, const oracle_line *ln, int c, double lam)
{
    const double lc = ln->lambda0 * (1.0 + par[3] / ORACLE_C_KMS);
    const double dlb = ORACLE_ZEEMAN_K * ln->lambda0 * ln->lambda0 * par[0];
    return (lam - lc - ln->shift[c] * dlb) / par[4];
}

/* One profile: out [4][L].  With par0 != NULL, each component's Faddeeva
 * value is taken to first order about its value at par0:
 *   w(z) ~ w(z0) + w'(z0) (z - z0),  w'(z) = -2 z w(z) + 2 i / sqrt(pi),
 * z = v + i a of the component at par, z0 at par0 (the derivative of the
 * Faddeeva function follows from its differential equation). */
static void synth_one_from(const double *par0, const double *par, double mu,
                           const oracle_line *lines, int nlines, int L, double *out)
{
    const double a = par[5];
    int off = 0;
    for (int l = 0; l < nlines; ++l) {
        const oracle_line *ln = &lines[l];
        for (int j = 0; j < ln->nlam; ++j) {
            const double lam = ln->start + (double)j * ln->step;
            double phi[3] = {0.0, 0.0, 0.0}, psi[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < ln->ncomp; ++c) {
                const double v = component_v(par, ln, c, lam);
                double H, Lf;
                if (!par0) {
                    oracle_faddeeva(v, a, &H, &Lf);
                } else {
                    const double v0 = component_v(par0, ln, c, lam), a0 = par0[5];
                    double H0, L0;
                    oracle_faddeeva(v0, a0, &H0, &L0);
                    const double complex z0 = v0 + I * a0, w0 = H0 + I * L0;
                    const double complex dw = -2.0 * z0 * w0 + 2.0 * I / sqrt(M_PI);
                    const double complex w = w0 + dw * ((v - v0) + I * (a - a0));
                    H = creal(w);
                    Lf = cimag(w);
                }
                phi[ln->q[c] + 1] += ln->strength[c] * H;
                psi[ln->q[c] + 1] += ln->strength[c] * Lf;
            }
            double st[4];
            stokes_from_profiles(par, mu, phi, psi, st);
            for (int s4 = 0; s4 < 4; ++s4)
                out[s4 * L + off + j] = st[s4];
        }
        off += ln->nlam;
    }
}

static void synth_one(const double *par, double mu, const oracle_line *lines, int nlines, int L,
                      double *out)
{
    synth_one_from(NULL, par, mu, lines, nlines, L, out);
}

void oracle_me_synth_lin(const double *par0, const double *par, double mu,
                         const oracle_line *lines, int nlines, double *out)
{
    synth_one_from(par0, par, mu, lines, nlines, total_samples(lines, nlines), out);
}

void oracle_me_synth(const double *par, int64_t n, const oracle_line *lines, int nlines,
                     const double *mu, double *out)
{
    const int L = total_samples(lines, nlines);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i)
        synth_one(par + i * ORACLE_NPAR, mu ? mu[i] : 1.0, lines, nlines, L, out + i * 4 * L);
}

/* chi-square of one model against one pixel's observation (Sec. 5, merit
 * function; weights w_i = 1/sigma_i, constant over wavelength). */
static double chi2_one(const double *par, double mu, const oracle_line *lines, int nlines, int L,
                       const double *obs, const double *sigma, double *scratch)
{
    synth_one(par, mu, lines, nlines, L, scratch);
    const double nu = 4.0 * L - ORACLE_NPAR;
    double s = 0.0;
    for (int st = 0; st < 4; ++st)
        for (int j = 0; j < L; ++j) {
            const double r = (obs[st * L + j] - scratch[st * L + j]) / sigma[st];
            s += r * r;
        }
    return s / nu;
}

void oracle_chi2(const double *par, int64_t npix, int pop, const oracle_line *lines, int nlines,
                 const double *obs, const double *sigma, const double *mu, double *chi2)
{
    const int L = total_samples(lines, nlines);
#pragma omp parallel
    {
        double *scratch = (double *)malloc(sizeof(double) * 4 * (size_t)L);
#pragma omp for schedule(dynamic, 1) collapse(2)
        for (int64_t p = 0; p < npix; ++p)
            for (int i = 0; i < pop; ++i)
                chi2[p * pop + i] = chi2_one(par + (p * pop + i) * ORACLE_NPAR, mu ? mu[p] : 1.0,
                                             lines, nlines, L, obs + p * 4 * L, sigma + p * 4,
                                             scratch);
        free(scratch);
    }
}

/* Used by the GA driver in oracle_ga.c. */
double oracle__chi2_single(const double *par, double mu, const oracle_line *lines, int nlines,
                           const double *obs, const double *sigma, double *scratch)
{
    return chi2_one(par, mu, lines, nlines, total_samples(lines, nlines), obs, sigma, scratch);
}

int oracle__total_samples(const oracle_line *lines, int nlines)
{
    return total_samples(lines, nlines);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
