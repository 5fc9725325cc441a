// Device building blocks of the gfx950 inversion kernels: counter-based
// random stream, Faddeeva approximations, Milne-Eddington synthesis and the
// genetic operators.  Section numbers refer to Harker & Mighell, "A
// GPU-Computing Approach to Solar Stokes Profile Inversion".
//
// Mapping: one workgroup per pixel, one GA individual per lane.  Every lane
// walks the same wavelength/component loop (trip counts are wavefront
// uniform, component tables live in kernel arguments and are read with
// scalar loads), the pixel's observation is broadcast from LDS, so the inner
// loop is pure VALU work on per-lane registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/genesis.h"
#include "voigt_rational.h"
#include "weideman36.h"

namespace genesis {

constexpr double kCkms = 299792.458;      // speed of light [km/s]
constexpr double kZeeman = 4.6686e-13;    // Delta lambda_B / (lambda0^2 B) [1/(A G)]
constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------------
// Lines as the kernels see them.  Components are grouped b (q = -1),
// p (q = 0), r (q = +1) so that the inner loops need no per-component branch.
template <typename Real>
struct DevLine {
    Real off0;     // first sample minus lambda0 [A]
    Real step;     // sample spacing [A]
    Real dop_kms;  // lambda0 / c [A per km/s]
    Real zee_G;    // 4.6686e-13 lambda0^2 [A per G]
    int32_t nlam, off, nb, np, nr, pad_;
    Real s[GENESIS_MAX_COMP];  // shift in units of Delta lambda_B
    Real w[GENESIS_MAX_COMP];  // strength
};

template <typename Real>
struct DevLines {
    int32_t nlines, L;
    DevLine<Real> l[GENESIS_MAX_LINES];
};

template <typename Real>
struct alignas(4 * sizeof(Real)) Vec4 {
    Real x, y, z, w;
};

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Word n of the stream
// (seed, pixel, generation, individual, purpose) is component n % 4 of the
// block with counter (pixel, generation, individual, purpose << 24 | n / 4).
struct Key {
    uint32_t k0, k1;
};

__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        Key key)
{
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t pick(uint4 b, uint32_t i)
{
    return i == 0 ? b.x : i == 1 ? b.y : i == 2 ? b.z : b.w;
}

// uniform integer in [0, m]: multiply-high, no rejection
__device__ __forceinline__ uint32_t uniform_upto(uint32_t word, uint32_t m)
{
    return (uint32_t)(((uint64_t)word * ((uint64_t)m + 1u)) >> 32);
}

enum Purpose : uint32_t { kInit = 0, kTournament = 1, kCross = 2, kMutate = 3 };

// ------------------------------------------------------------------------
// Faddeeva function w(v + i a) -> (H, L) = (Re w, Im w) (Sec. 5: Voigt and
// Faraday-Voigt profiles).
//
// FP32: w = P(Z)/Q(Z), Z = a - i v, real coefficients (deg 6 / 7, the
// degrees of Hui, Armstrong & Wray's approximation), fitted on Re Z = 0
// (maximum error 1.5e-7, which bounds the error for every a >= 0).
// Expanding around Z = a once per individual gives polynomials in u = v^2:
//   P(a - i v) = EP(u) - i v OP(u),  Q(a - i v) = EQ(u) - i v OQ(u),
// so one profile evaluation costs 11 FMAs of Horner plus one reciprocal:
//   H = (EP EQ + u OP OQ) / (EQ^2 + u OQ^2),  L = v (EP OQ - OP EQ) / (...).
constexpr int kNP = GENESIS_VR_NP, kNQ = GENESIS_VR_NQ;  // coefficient counts of P, Q
constexpr int kEP = (kNP + 1) / 2, kOP = kNP / 2;        // even / odd parts of P in u
constexpr int kEQ = (kNQ + 1) / 2, kOQ = kNQ / 2;        // even / odd parts of Q in u

struct VoigtF32 {
    float ep[kEP], op[kOP], eq[kEQ], oq[kOQ];
};

// Coefficients of c(x + a) = sum_k r_k x^k: r_k = sum_{m >= k} C(m, k) c_m a^(m-k),
// each evaluated by its own Horner scheme in a (few live registers).
template <int N>
struct ShiftTable {
    double t[N][N];  // t[k][m - k] = C(m, k) c_m
};

template <int N>
constexpr ShiftTable<N> shift_table(const double (&c)[N])
{
    ShiftTable<N> s{};
    for (int k = 0; k < N; ++k) {
        double binom = 1.0;  // C(m, k) for m = k
        for (int m = k; m < N; ++m) {
            s.t[k][m - k] = binom * c[m];
            binom = binom * (double)(m + 1) / (double)(m + 1 - k);
        }
    }
    return s;
}

constexpr double kVrP[GENESIS_VR_NP] = {GENESIS_VR_P_INIT};
constexpr double kVrQ[GENESIS_VR_NQ] = {GENESIS_VR_Q_INIT};
constexpr ShiftTable<GENESIS_VR_NP> kShiftP = shift_table(kVrP);
constexpr ShiftTable<GENESIS_VR_NQ> kShiftQ = shift_table(kVrQ);

template <int N>
__device__ __forceinline__ float shifted(const ShiftTable<N> &s, int k, double a)
{
    double r = s.t[k][N - 1 - k];
#pragma unroll
    for (int i = N - 2 - k; i >= 0; --i)
        r = fma(r, a, s.t[k][i]);
    return (float)r;
}

__device__ __forceinline__ VoigtF32 voigt_setup_f32(double a)
{
    VoigtF32 c;
    // (-i v)^(2m) = (-1)^m u^m ; (-i v)^(2m+1) = -i v (-1)^m u^m
#pragma unroll
    for (int m = 0; m < kEP; ++m)
        c.ep[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftP, 2 * m, a);
#pragma unroll
    for (int m = 0; m < kOP; ++m)
        c.op[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftP, 2 * m + 1, a);
#pragma unroll
    for (int m = 0; m < kEQ; ++m)
        c.eq[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftQ, 2 * m, a);
#pragma unroll
    for (int m = 0; m < kOQ; ++m)
        c.oq[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftQ, 2 * m + 1, a);
    return c;
}

template <int N>
__device__ __forceinline__ float horner(const float (&c)[N], float u)
{
    float r = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k)
        r = fmaf(r, u, c[k]);
    return r;
}

// h += w H(v), l += w L(v): the Horner schemes, one reciprocal, and the
// strength folded into the reciprocal; u OQ is shared by numerator and
// denominator.
__device__ __forceinline__ void voigt_acc_f32(const VoigtF32 &c, float v, float w, float &h,
                                              float &l)
{
    const float u = v * v;
    const float ep = horner(c.ep, u);
    const float op = horner(c.op, u);
    const float eq = horner(c.eq, u);
    const float oq = horner(c.oq, u);
    const float uoq = u * oq;
    const float wr = w * __builtin_amdgcn_rcpf(fmaf(eq, eq, oq * uoq));
    h = fmaf(fmaf(ep, eq, op * uoq), wr, h);
    l = fmaf(v * fmaf(ep, oq, -(op * eq)), wr, l);
}

// FP64: Weideman's expansion with the N coefficients c and parameter WL.
template <int N>
__device__ __forceinline__ void weideman_w(const double (&c)[N], double WL, double a, double v,
                                           double &H, double &L)
{
    // d = L - i z with z = v + i a  ->  d = (WL + a) - i v ; r = 1/d
    const double dr = WL + a, di = -v;
    const double inv = 1.0 / fma(dr, dr, di * di);
    const double rr = dr * inv, ri = -di * inv;
    // Z = (L + i z) r = ((WL - a) + i v) r
    const double nr = WL - a, ni = v;
    const double Zr = fma(nr, rr, -(ni * ri));
    const double Zi = fma(nr, ri, ni * rr);
    double pr = c[N - 1], pi = 0.0;
#pragma unroll
    for (int n = N - 2; n >= 0; --n) {
        const double tr = fma(pr, Zr, fma(-pi, Zi, c[n]));
        const double ti = fma(pr, Zi, pi * Zr);
        pr = tr;
        pi = ti;
    }
    // w = r (2 p r + 1/sqrt(pi))
    const double tr = fma(2.0, fma(pr, rr, -(pi * ri)), 0.56418958354775628695);
    const double ti = 2.0 * fma(pr, ri, pi * rr);
    H = fma(tr, rr, -(ti * ri));
    L = fma(tr, ri, ti * rr);
}

// The FP64 kernels' Faddeeva function: N = 36 (error ~2e-15).
__device__ __forceinline__ void voigt_f64(double a, double v, double &H, double &L)
{
    weideman_w(genesis_wd36_c, GENESIS_WD36_L, a, v, H, L);
}

__device__ __forceinline__ void voigt_acc_f64(double a, double v, double w, double &h, double &l)
{
    double H, L;
    voigt_f64(a, v, H, L);
    h = fma(w, H, h);
    l = fma(w, L, l);
}

// ------------------------------------------------------------------------
// Per-individual constants of the Milne-Eddington model (Sec. 5).
template <typename Real>
struct Model;

template <>
struct Model<float> {
    float B, inv_dop, vlos;
    float cI1, cI2, cQ, cU, cV, c2;  // eta0/2 folded in; c2 = cQ^2 + cU^2
    float S0, muS1;
    VoigtF32 vc;
};

template <>
struct Model<double> {
    double B, inv_dop, vlos, a;
    double cI1, cI2, cQ, cU, cV, c2;
    double S0, muS1;
};

// Geometry factors of the propagation matrix (absorption eta and
// magneto-optical rho share them):
//   eta_I = eta0/2 [phi_p sin^2(g) + (phi_b + phi_r)(1 + cos^2(g))/2]
//   eta_Q = eta0/2 [phi_p - (phi_b + phi_r)/2] sin^2(g) cos(2 chi)
//   eta_U = eta0/2 [phi_p - (phi_b + phi_r)/2] sin^2(g) sin(2 chi)
//   eta_V = eta0/2 (phi_r - phi_b) cos(g)
template <typename Real>
__device__ __forceinline__ void model_common(const double (&p)[GENESIS_NPAR], double mu,
                                             Model<Real> &m)
{
    const double g = p[1] * (kPi / 180.0), chi = p[2] * (kPi / 180.0);
    double sg, cg, s2x, c2x;
    sincos(g, &sg, &cg);
    sincos(2.0 * chi, &s2x, &c2x);
    const double h = 0.5 * p[6];
    const double sg2 = sg * sg;
    m.B = (Real)p[0];
    m.inv_dop = (Real)(1.0 / p[4]);
    m.vlos = (Real)p[3];
    m.cI1 = (Real)(h * sg2);
    m.cI2 = (Real)(0.5 * h * (1.0 + cg * cg));
    m.cQ = (Real)(h * sg2 * c2x);
    m.cU = (Real)(h * sg2 * s2x);
    m.cV = (Real)(h * cg);
    m.c2 = (Real)(h * sg2 * h * sg2);
    m.S0 = (Real)p[7];
    m.muS1 = (Real)(mu * p[8]);
}

__device__ __forceinline__ void model_setup(const double (&p)[GENESIS_NPAR], double mu,
                                            Model<float> &m)
{
    // FP32 model: angles, geometry and Voigt coefficients in FP32 after the
    // FP64 decode (keeps the per-individual set-up register-light)
    float sg, cg, s2x, c2x;
    sincosf((float)(p[1] * (kPi / 180.0)), &sg, &cg);
    sincosf((float)(p[2] * (kPi / 90.0)), &s2x, &c2x);
    const float h = 0.5f * (float)p[6];
    const float sg2 = sg * sg;
    m.B = (float)p[0];
    m.inv_dop = (float)(1.0 / p[4]);
    m.vlos = (float)p[3];
    m.cI1 = h * sg2;
    m.cI2 = 0.5f * h * fmaf(cg, cg, 1.0f);
    m.cQ = h * sg2 * c2x;
    m.cU = h * sg2 * s2x;
    m.cV = h * cg;
    m.c2 = (h * sg2) * (h * sg2);
    m.S0 = (float)p[7];
    m.muS1 = (float)(mu * p[8]);
    m.vc = voigt_setup_f32(p[5]);
}

__device__ __forceinline__ void model_setup(const double (&p)[GENESIS_NPAR], double mu,
                                            Model<double> &m)
{
    model_common(p, mu, m);
    m.a = p[5];
}

__device__ __forceinline__ void profile_acc(const Model<float> &m, float v, float w, float &h,
                                            float &l)
{
    voigt_acc_f32(m.vc, v, w, h, l);
}

__device__ __forceinline__ void profile_acc(const Model<double> &m, double v, double w,
                                            double &h, double &l)
{
    voigt_acc_f64(m.a, v, w, h, l);
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Components of one Zeeman group at wavelength offset x0 (reduced units):
// accumulate strength-weighted H and L.  N >= 0: compile-time count (the
// component table then sits in scalar registers for the whole line);
// N < 0: runtime count n.
template <int N, typename Real>
__device__ __forceinline__ void group(const Model<Real> &m, const DevLine<Real> &ln, int c0,
                                      int n, Real x0, Real zb, Real &h, Real &l)
{
    if constexpr (N >= 0) {
#pragma unroll
        for (int c = 0; c < N; ++c)
            profile_acc(m, fma(-ln.s[c0 + c], zb, x0), ln.w[c0 + c], h, l);
    } else {
        for (int c = c0; c < c0 + n; ++c)
            profile_acc(m, fma(-ln.s[c], zb, x0), ln.w[c], h, l);
    }
}

// Stokes vector at one wavelength from the strength-weighted group profiles:
// Unno-Rachkovsky closed form with k = 1 + eta_I,
//   Pi = eta.rho, Delta = k^2 (k^2 - |eta|^2 + |rho|^2) - Pi^2,
//   I = S0 + mu S1 k (k^2 + |rho|^2) / Delta,
//   Q = -mu S1 [k^2 eta_Q + k (eta_V rho_U - eta_U rho_V) + rho_Q Pi] / Delta
//   (U, V by cyclic permutation Q -> U -> V),
// i.e. S0 e + mu S1 K^-1 e for K = 1 + eta0 Phi.  Because eta_Q, eta_U,
// rho_Q, rho_U share the azimuth factors (eta_Q = cQ h_t, rho_Q = cQ l_t,
// eta_U = cU h_t, rho_U = cU l_t), eta_U rho_Q - eta_Q rho_U = 0 and, with
// c2 = cQ^2 + cU^2, X = eta_V l_t - h_t rho_V, A = k^2 h_t + l_t Pi:
//   |eta|^2 = c2 h_t^2 + eta_V^2, |rho|^2 = c2 l_t^2 + rho_V^2,
//   Pi = c2 h_t l_t + eta_V rho_V,
//   Q = -mu S1 (cQ A + cU k X) / Delta, U = -mu S1 (cU A - cQ k X) / Delta,
//   V = -mu S1 (k^2 eta_V + rho_V Pi) / Delta.
template <typename Real, typename M>
__device__ __forceinline__ void unno_rachkovsky(const M &m, Real hb, Real lb, Real hp,
                                                Real lp, Real hr, Real lr, Real &I, Real &Q,
                                                Real &U, Real &V)
{
    const Real hs = hb + hr, ls_ = lb + lr;
    const Real ht = fma((Real)-0.5, hs, hp), lt = fma((Real)-0.5, ls_, lp);
    const Real eI = fma(m.cI1, hp, m.cI2 * hs);
    const Real eV = m.cV * (hr - hb), rV = m.cV * (lr - lb);
    const Real k = (Real)1 + eI;
    const Real k2 = k * k;
    const Real e2 = fma(ht * ht, m.c2, eV * eV);
    const Real r2 = fma(lt * lt, m.c2, rV * rV);
    const Real Pi = fma(ht * lt, m.c2, eV * rV);
    const Real D = fma(k2, k2 - e2 + r2, -(Pi * Pi));
    const Real nrD = -(m.muS1 * recip(D));
    I = fma(-(k * (k2 + r2)), nrD, m.S0);
    const Real X = fma(eV, lt, -(ht * rV));
    const Real kX = k * X;
    const Real A = fma(k2, ht, lt * Pi);
    Q = fma(m.cQ, A, m.cU * kX) * nrD;
    U = fma(m.cU, A, -(m.cQ * kX)) * nrD;
    V = fma(k2, eV, rV * Pi) * nrD;
}

// Samples j0 .. j1-1 of one line, handing (j, I, Q, U, V) to `sink`.
template <int NB, int NP, int NR, typename Real, typename Sink>
__device__ __forceinline__ void synth_line(const Model<Real> &m, const DevLine<Real> &ln,
                                           Sink &sink, int j0, int j1)
{
    const Real xb = (ln.off0 - m.vlos * ln.dop_kms) * m.inv_dop;
    const Real xs = ln.step * m.inv_dop;
    const Real zb = ln.zee_G * m.B * m.inv_dop;
    const int nb = NB >= 0 ? NB : ln.nb, np = NP >= 0 ? NP : ln.np;
    const int nr = NR >= 0 ? NR : ln.nr;
    for (int j = j0; j < j1; ++j) {
        const Real x0 = fma((Real)j, xs, xb);
        Real hb = 0, lb = 0, hp = 0, lp = 0, hr = 0, lr = 0;
        group<NB>(m, ln, 0, nb, x0, zb, hb, lb);
        group<NP>(m, ln, nb, np, x0, zb, hp, lp);
        group<NR>(m, ln, nb + np, nr, x0, zb, hr, lr);
        Real I, Q, U, V;
        unno_rachkovsky(m, hb, lb, hp, lp, hr, lr, I, Q, U, V);
        sink(ln.off + j, I, Q, U, V);
    }
}

// The two Zeeman patterns of the Fe I 6302 pair (a triplet and the 4 + 4 + 4
// pattern of 6301.5) get compile-time component counts.
template <typename Real, typename Sink>
__device__ __forceinline__ void synth_line_range(const Model<Real> &m, const DevLine<Real> &ln,
                                                 Sink &sink, int j0, int j1)
{
    if (ln.nb == 1 && ln.np == 1 && ln.nr == 1)
        synth_line<1, 1, 1>(m, ln, sink, j0, j1);
    else if (ln.nb == 4 && ln.np == 4 && ln.nr == 4)
        synth_line<4, 4, 4>(m, ln, sink, j0, j1);
    else
        synth_line<-1, -1, -1>(m, ln, sink, j0, j1);
}

// Every line.
template <typename Real, typename Sink>
__device__ __forceinline__ void synthesize(const Model<Real> &m, const DevLines<Real> &ls,
                                           Sink &sink)
{
    for (int l = 0; l < ls.nlines; ++l) {
        const DevLine<Real> &ln = ls.l[l];
        synth_line_range(m, ln, sink, 0, ln.nlam);
    }
}

// Stokes vector of one model at sample jj of one line (used where each lane
// owns a wavelength instead of an individual).
// The three group profiles (h, l of blue, pi, red) of one model at sample jj.
// They depend on the model only through B, v_los, the Doppler width and the
// damping.
template <typename Real>
__device__ __forceinline__ void profiles_at(const Model<Real> &m, const DevLine<Real> &ln, int jj,
                                            Real (&pr)[6])
{
    const Real xb = (ln.off0 - m.vlos * ln.dop_kms) * m.inv_dop;
    const Real x0 = fma((Real)jj, ln.step * m.inv_dop, xb);
    const Real zb = ln.zee_G * m.B * m.inv_dop;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        pr[i] = 0;
    group<-1>(m, ln, 0, ln.nb, x0, zb, pr[0], pr[1]);
    group<-1>(m, ln, ln.nb, ln.np, x0, zb, pr[2], pr[3]);
    group<-1>(m, ln, ln.nb + ln.np, ln.nr, x0, zb, pr[4], pr[5]);
}

template <typename Real>
__device__ __forceinline__ void stokes_at(const Model<Real> &m, const DevLine<Real> &ln, int jj,
                                          Real &I, Real &Q, Real &U, Real &V)
{
    Real pr[6];
    profiles_at(m, ln, jj, pr);
    unno_rachkovsky(m, pr[0], pr[1], pr[2], pr[3], pr[4], pr[5], I, Q, U, V);
}

// chi-square accumulator against an observation staged in LDS as
// [L] x (I, Q, U, V): per-Stokes sums of squared residuals, combined with the
// weights 1/sigma^2 at the end (Sec. 5 merit function).
template <typename Real>
struct Chi2Sink {
    const Vec4<Real> *obs;
    Real sI, sQ, sU, sV;
    __device__ __forceinline__ void operator()(int j, Real I, Real Q, Real U, Real V)
    {
        const Vec4<Real> o = obs[j];
        const Real dI = o.x - I, dQ = o.y - Q, dU = o.z - U, dV = o.w - V;
        sI = fma(dI, dI, sI);
        sQ = fma(dQ, dQ, sQ);
        sU = fma(dU, dU, sU);
        sV = fma(dV, dV, sV);
    }
};

template <typename Real>
__device__ __forceinline__ Real chi2_of(const Model<Real> &m, const DevLines<Real> &ls,
                                        const Vec4<Real> *obs_lds, const Real (&w2)[4],
                                        Real inv_nu)
{
    Chi2Sink<Real> s{obs_lds, 0, 0, 0, 0};
    synthesize(m, ls, s);
    return fma(w2[0], s.sI, fma(w2[1], s.sQ, fma(w2[2], s.sU, w2[3] * s.sV))) * inv_nu;
}

// ------------------------------------------------------------------------
// Decoding operator E^-1 (Sec. 3): p = lo + (hi - lo) g / 65535, in FP64.
struct Bounds {
    double lo[GENESIS_NPAR], span[GENESIS_NPAR];
};

__device__ __forceinline__ void decode(const uint32_t (&g)[GENESIS_NPAR], const Bounds &b,
                                       double (&p)[GENESIS_NPAR])
{
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        p[j] = b.lo[j] + b.span[j] * (double)g[j] / 65535.0;
}

// ------------------------------------------------------------------------
// Genetic operators (Sec. 3; genes as 16-bit integers, Sec. 4.2).
struct GaConst {
    int32_t pop, k;
    uint64_t thr_cross;          // crossover iff word < thr_cross (thr in [0, 2^32])
    uint32_t mut_thr[16];        // bit k (0 = MSB) flips iff 16-bit uniform < mut_thr[k]
    Key key;
    uint32_t pixel_base;
    int32_t n_seeded, seed_jitter;
    const float *seed_params;    // [npix][seed_sets][9] first guesses, or nullptr
    int32_t seed_sets;           // first guesses per pixel (>= 1)
    int32_t init_mode;           // 0 Philox-uniform genes, 1 Sobol points
    int32_t restart_every;       // 0: no restarts
    const float *pixel_bounds;   // [npix][2][9] per-pixel boxes (lo, hi), or nullptr
};

enum : uint32_t { kSobolShift = 4, kSeedJitter = 5 };

// ------------------------------------------------------------------------
// Sobol' points (Sobol' 1967; the construction of Bratley & Fox 1988) for
// the initial population and the restarts of Sec. 5.6.  Dimension 0 is the
// base-2 van der Corput sequence; dimension d >= 1 uses the d-th primitive
// polynomial over GF(2) in order of degree and then of value, with initial
// direction numbers m_1 = ... = m_s = 1 (odd and below 2^k, as required),
// and m_k = m_{k-s} ^ (m_{k-s} << s) ^ sum_{i=1}^{s-1} a_i (m_{k-i} << i)
// for p(x) = x^s + a_1 x^(s-1) + ... + a_(s-1) x + 1.  Point n, coordinate d:
// the XOR of V_k = m_k << (32 - k) over the set bits k - 1 of n.  The tables
// are built at compile time from these definitions.
struct SobolTable {
    uint32_t poly[GENESIS_NPAR];         // polynomial bits (x^s ... 1); dimension 0 unused
    uint32_t v[GENESIS_NPAR][32];        // V_k, k = 1 .. 32
};

constexpr uint32_t gf2_mulmod(uint32_t a, uint32_t b, uint32_t p, int deg)
{
    uint32_t r = 0;
    for (int i = 0; i < deg; ++i) {
        if (b & 1u)
            r ^= a;
        b >>= 1;
        a <<= 1;
        if (a & (1u << deg))
            a ^= p;
    }
    return r;
}

constexpr uint32_t gf2_xpow(uint64_t e, uint32_t p, int deg)
{
    uint32_t r = 1, b = deg > 1 ? 2u : (2u ^ p);  // x mod p
    while (e) {
        if (e & 1u)
            r = gf2_mulmod(r, b, p, deg);
        b = gf2_mulmod(b, b, p, deg);
        e >>= 1;
    }
    return r;
}

// p of degree deg with p(0) = 1 is primitive iff x has order 2^deg - 1 mod p.
constexpr bool gf2_primitive(uint32_t p, int deg)
{
    const uint64_t n = (1ull << deg) - 1;
    if (gf2_xpow(n, p, deg) != 1u)
        return false;
    uint64_t m = n;
    for (uint64_t q = 2; q * q <= m; ++q) {
        if (m % q)
            continue;
        if (gf2_xpow(n / q, p, deg) == 1u)
            return false;
        while (m % q == 0)
            m /= q;
    }
    if (m > 1 && m != n && gf2_xpow(n / m, p, deg) == 1u)
        return false;
    if (m == n && n > 1 && gf2_xpow(1, p, deg) == 1u)
        return false;
    return true;
}

constexpr SobolTable make_sobol()
{
    SobolTable t{};
    for (int k = 1; k <= 32; ++k)
        t.v[0][k - 1] = 1u << (32 - k);
    int d = 1;
    for (int deg = 1; d < GENESIS_NPAR; ++deg)
        for (uint32_t p = (1u << deg) | 1u; p < (2u << deg) && d < GENESIS_NPAR; p += 2)
            if (gf2_primitive(p, deg))
                t.poly[d++] = p;
    for (d = 1; d < GENESIS_NPAR; ++d) {
        const uint32_t p = t.poly[d];
        int s = 0;
        while ((p >> (s + 1)) != 0)
            ++s;
        uint32_t m[33] = {};
        for (int k = 1; k <= 32; ++k) {
            if (k <= s) {
                m[k] = 1u;
            } else {
                uint32_t x = m[k - s] ^ (m[k - s] << s);
                for (int i = 1; i < s; ++i)
                    if ((p >> (s - i)) & 1u)
                        x ^= m[k - i] << i;
                m[k] = x;
            }
            t.v[d][k - 1] = m[k] << (32 - k);
        }
    }
    return t;
}

constexpr SobolTable kSobol = make_sobol();

__device__ __forceinline__ uint32_t sobol_coord(int d, uint32_t n)
{
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k)
        if ((n >> k) & 1u)
            x ^= kSobol.v[d][k];
    return x;
}

// Genes of Sobol point n for pixel pix: the point's coordinates XORed with a
// per-pixel digital shift (stream purpose 4, individual 0), top 16 bits.
__device__ __forceinline__ void sobol_genes(uint32_t pix, uint32_t n, const Key &key,
                                            uint32_t (&g)[GENESIS_NPAR])
{
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        const uint4 w = philox(pix, 0u, 0u, (kSobolShift << 24) | (uint32_t)blk, key);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * blk + q;
            if (j < GENESIS_NPAR)
                g[j] = (sobol_coord(j, n) ^ ws[q]) >> 16;
        }
    }
}

// The nine genes of individual i of pixel p (call-local index) in generation
// 0: random (stream purpose 0) or Sobol point i (init_mode 1); for
// i < n_seeded, every parameter whose first guess is not NaN instead takes
// the encoded guess i mod S of the pixel's S = seed_sets guesses (exact for
// i < S, integer-jittered for i >= S, stream purpose 5).
__device__ __forceinline__ void initial_genes(uint32_t pix, int64_t p, int i, const GaConst &ga,
                                              const Bounds &b, uint32_t (&g)[GENESIS_NPAR])
{
    // the unseeded genes of individual i first
    if (ga.init_mode == 1) {
        sobol_genes(pix, (uint32_t)i, ga.key, g);
    } else {
#pragma unroll
        for (int blk = 0; blk < 3; ++blk) {
            const uint4 w = philox(pix, 0u, (uint32_t)i, (kInit << 24) | (uint32_t)blk, ga.key);
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * blk + q < GENESIS_NPAR)
                    g[4 * blk + q] = ws[q] >> 16;
        }
    }
    if (!(i < ga.n_seeded && ga.seed_params))
        return;
    const int S = ga.seed_sets;
    const float *guess = ga.seed_params + (p * S + i % S) * GENESIS_NPAR;
    // seeded slot: every parameter with a finite first guess takes its code
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        const uint4 w = philox(pix, 0u, (uint32_t)i, (kSeedJitter << 24) | (uint32_t)blk, ga.key);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * blk + q;
            if (j >= GENESIS_NPAR)
                continue;
            const float sp = guess[j];
            if (isnan(sp))
                continue;
            double u = ((double)sp - b.lo[j]) / (b.span[j] > 0.0 ? b.span[j] : 1.0);
            u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
            int v = (int)floor(u * 65535.0 + 0.5);
            if (i >= S) {
                v += (int)uniform_upto(ws[q], 2u * (uint32_t)ga.seed_jitter) - ga.seed_jitter;
                v = v < 0 ? 0 : (v > 65535 ? 65535 : v);
            }
            g[j] = (uint32_t)v;
        }
    }
}

// fitness order: NaN reads as +infinity, ties go to the lower index
template <typename Real>
__device__ __forceinline__ Real fit_key(Real f)
{
    return isnan(f) ? (Real)INFINITY : f;
}

template <typename Real>
__device__ __forceinline__ bool before(Real fa, int ia, Real fb, int ib)
{
    return fa < fb || (fa == fb && ia < ib);
}

// Tournament of k distinct contestants drawn by Floyd's algorithm from the
// words which*k .. which*k + k - 1 of stream (pixel, gen, pair, 1).
template <typename Real>
__device__ __forceinline__ int tournament(const Real *fit_s, int pop, int k, Key key,
                                          uint32_t pixel, uint32_t gen, uint32_t pair, int which)
{
    int chosen[GENESIS_MAX_K];
    int best = 0;
    Real bestf = (Real)INFINITY;
    uint32_t blk_id = 0xFFFFFFFFu;
    uint4 blk = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < GENESIS_MAX_K; ++i) {
        if (i < k) {
            const uint32_t n = (uint32_t)(which * k + i);
            if ((n >> 2) != blk_id) {
                blk_id = n >> 2;
                blk = philox(pixel, gen, pair, (kTournament << 24) | blk_id, key);
            }
            const int j = pop - k + i;
            int t = (int)uniform_upto(pick(blk, n & 3u), (uint32_t)j);
            bool seen = false;
#pragma unroll
            for (int c = 0; c < GENESIS_MAX_K; ++c)
                if (c < i && chosen[c] == t)
                    seen = true;
            t = seen ? j : t;
            chosen[i] = t;
            const Real f = fit_key(fit_s[t]);
            if (i == 0 || before(f, t, bestf, best)) {
                best = t;
                bestf = f;
            }
        }
    }
    return best;
}

__device__ __forceinline__ uint32_t first_parent_mask(int j, int x)
{
    const int lo = j * 16;
    if (x >= lo + 16)
        return 0xFFFFu;
    if (x <= lo)
        return 0u;
    return (0xFFFFu << (16 - (x - lo))) & 0xFFFFu;
}

// Child of slot c >= 1 (child (c-1)%2 of pair (c-1)/2) of generation gen.
// genes_s is the parent population in LDS as [9][pop]; `out` receives
// out.meta(parent A, parent B, crossover point) and out.gene(j, gene, mask).
template <typename Real, typename Out>
__device__ __forceinline__ void make_child(int c, uint32_t pixel, uint32_t gen,
                                           const Real *fit_s, const uint16_t *genes_s,
                                           const GaConst &ga, Out &out)
{
    const int pop = ga.pop;
    const uint32_t pair = (uint32_t)((c - 1) >> 1);
    const bool second = ((c - 1) & 1) != 0;
    const int A = tournament(fit_s, pop, ga.k, ga.key, pixel, gen, pair, 0);
    const int B = tournament(fit_s, pop, ga.k, ga.key, pixel, gen, pair, 1);
    const uint4 cw = philox(pixel, gen, pair, kCross << 24, ga.key);
    const bool cross = (uint64_t)cw.x < ga.thr_cross;
    const int x = cross ? 1 + (int)uniform_upto(cw.y, GENESIS_NPAR * 16 - 2) : 0;
    const int first = second ? B : A, other = second ? A : B;
    out.meta(A, B, x);
#pragma unroll 1
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        const uint32_t m = cross ? first_parent_mask(j, x) : 0xFFFFu;
        const uint32_t g1 = genes_s[j * pop + first], g2 = genes_s[j * pop + other];
        const uint32_t child = (g1 & m) | (g2 & (~m & 0xFFFFu));
        // mutation: block 2j + h of stream (pixel, gen, c, 3) holds the 16-bit
        // uniforms of bits 8h .. 8h + 7 of gene j (low half of a word first)
        uint32_t mk = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint4 b = philox(pixel, gen, (uint32_t)c,
                                   (kMutate << 24) | (uint32_t)(2 * j + h), ga.key);
            const uint32_t wds[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kb = 8 * h + q;
                const uint32_t wd = wds[q >> 1];
                const uint32_t u16 = (q & 1) ? (wd >> 16) : (wd & 0xFFFFu);
                mk |= (u16 < ga.mut_thr[kb]) ? (1u << (15 - kb)) : 0u;
            }
        }
        out.gene(j, child ^ mk, mk);
    }
}

// Block-wide argmin of fit_s[0 .. pop) (NaN = +inf, ties to the lower index);
// every thread gets the result.  red_f/red_i: LDS scratch of one entry per
// wavefront.
template <typename Real>
__device__ __forceinline__ int block_argmin(const Real *fit_s, int pop, Real *red_f, int *red_i)
{
    const int tid = threadIdx.x;
    Real f = tid < pop ? fit_key(fit_s[tid]) : (Real)INFINITY;
    int idx = tid < pop ? tid : 0x7FFFFFFF;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const Real f2 = __shfl_xor(f, off);
        const int i2 = __shfl_xor(idx, off);
        if (before(f2, i2, f, idx)) {
            f = f2;
            idx = i2;
        }
    }
    if ((tid & 63) == 0) {
        red_f[tid >> 6] = f;
        red_i[tid >> 6] = idx;
    }
    __syncthreads();
    const int nw = (int)(blockDim.x >> 6);
    f = red_f[0];
    idx = red_i[0];
    for (int w = 1; w < nw; ++w)
        if (before(red_f[w], red_i[w], f, idx)) {
            f = red_f[w];
            idx = red_i[w];
        }
    return idx;
}

// Restarts (Sec. 5.6): after the evaluation of generation t, when
// restart_every > 0, t > 0, t < G and t is a multiple of restart_every, the
// worst nrep = pop / 2 individuals (fitness order of the tournaments: NaN
// last, ties to the lower index) are replaced by fresh Sobol points: the
// individual of rank pop - nrep + q takes point pop + (r - 1) nrep + q of
// the pixel's shifted sequence, r = t / restart_every.
__device__ __forceinline__ bool restart_due(const GaConst &ga, int t, int generations)
{
    return ga.restart_every > 0 && t > 0 && t < generations && t % ga.restart_every == 0;
}

template <typename Real>
__device__ __forceinline__ int fitness_rank(const Real *fit_s, int pop, int i)
{
    const Real fi = fit_key(fit_s[i]);
    int r = 0;
    for (int j = 0; j < pop; ++j)
        r += before(fit_key(fit_s[j]), j, fi, i) ? 1 : 0;
    return r;
}

// Genes of the restart replacement for an individual of rank `rank` at
// generation t; false if the individual is kept.
__device__ __forceinline__ bool restart_genes(const GaConst &ga, uint32_t pix, int t, int rank,
                                              uint32_t (&g)[GENESIS_NPAR])
{
    const int nrep = ga.pop / 2;
    const int q = rank - (ga.pop - nrep);
    if (q < 0)
        return false;
    const uint32_t r = (uint32_t)(t / ga.restart_every);
    sobol_genes(pix, (uint32_t)ga.pop + (r - 1u) * (uint32_t)nrep + (uint32_t)q, ga.key, g);
    return true;
}

}  // namespace genesis
