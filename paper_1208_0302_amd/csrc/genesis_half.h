// Reduced-precision synthesis: the Voigt and Faraday-Voigt profiles of every
// Zeeman component (Sec. 5) evaluated in packed FP16, two wavelengths per
// lane per instruction (v_pk_fma_f16), with the reduced wavelength formed in
// FP32, the Unno-Rachkovsky solution and the chi-square in FP32.
//
// FP16 rounding alone limits the profiles to a few 1e-3, so this path uses
// its own low-degree rational w = P(Z)/Q(Z) (voigt_rational_h.h: degree
// n-1 / n in Z = a - i v with n = 4, error 1.5e-4 for every damping) rather
// than the FP32 kernels' degree-7 one.  Per individual it gives
// H = NH(u)/D(u) and L = v NL(u)/D(u) with u = v^2, NH and NL of degree n-1
// and D of degree n.  Their values span many orders of magnitude over the
// line window, beyond FP16's range, so each is mapped to the compact variable
// t = 1/(1 + u/s) in (0, 1]:
//   X~(t) = t^n X(s (1 - t)/t) = sum_k x_k s^k (1 - t)^k t^(n - k),
// a degree-n polynomial in t whose ratio NH~/D~ is still H.  Numerators and
// denominator are scaled by the same factor 1/sqrt(D~(0) D~(1)), which keeps
// every coefficient at most 4.3 in magnitude for damping a <= 1, so FP16
// rounds each by at most 2e-3.  Per component and pair of wavelengths: 2 mixed-precision FMAs
// for v, 1 multiply and 1 FMA for t's denominator, 2 reciprocals, 3 n Horner
// FMAs, 2 reciprocals for 1/D~, and 4 operations to accumulate the
// strength-weighted H and L.  Simulated worst error of the FP16 evaluation
// over a in [0, 1], |v| <= 300: about 4.4e-3 in H and 2.7e-3 in L
// (1 = H(0, 0)).
#pragma once

#include "genesis_device.h"
#include "voigt_rational_h.h"

namespace genesis {

typedef _Float16 half_t;
typedef half_t h2 __attribute__((ext_vector_type(2)));

constexpr double kHalfS = 2.0;        // u scale of the compact variable
constexpr double kHalfMaxDamping = 1.0;

constexpr int kHNP = GENESIS_VRH_NP, kHNQ = GENESIS_VRH_NQ;  // coefficient counts of P, Q
constexpr int kHEP = (kHNP + 1) / 2, kHOP = kHNP / 2;          // even / odd parts in u
constexpr int kHEQ = (kHNQ + 1) / 2, kHOQ = kHNQ / 2;
constexpr double kVrhP[kHNP] = {GENESIS_VRH_P_INIT};
constexpr double kVrhQ[kHNQ] = {GENESIS_VRH_Q_INIT};
constexpr ShiftTable<kHNP> kShiftPH = shift_table(kVrhP);
constexpr ShiftTable<kHNQ> kShiftQH = shift_table(kVrhQ);

constexpr int kDegH = kHNQ - 1;  // degree n of D in u
constexpr int kNH = kDegH + 1;   // coefficients per compact polynomial

// T[m][k]: coefficient of t^m contributed by u^k, s^k C(k, i) (-1)^i with
// i = m - n + k, for k >= n - m.
struct TTable {
    double t[kNH][kNH];
};

constexpr TTable make_ttable()
{
    TTable T{};
    for (int m = 0; m <= kDegH; ++m)
        for (int k = kDegH - m; k <= kDegH; ++k) {
            const int i = m - kDegH + k;
            double binom = 1.0;
            for (int r = 0; r < i; ++r)
                binom = binom * (double)(k - r) / (double)(r + 1);
            double sk = 1.0;
            for (int r = 0; r < k; ++r)
                sk *= kHalfS;
            T.t[m][k] = sk * binom * ((i & 1) ? -1.0 : 1.0);
        }
    return T;
}

constexpr TTable kTT = make_ttable();

// Packed coefficients: nh~[0..n], nl~[0..n], d~[0..n] at index q of c[q / 2][q % 2].
struct VoigtH {
    h2 c[(3 * kNH + 1) / 2];
};

__device__ __forceinline__ void to_t(const float (&x)[kNH], float (&y)[kNH])
{
#pragma unroll
    for (int m = 0; m <= kDegH; ++m) {
        float s = 0.0f;
#pragma unroll
        for (int k = kDegH - m; k <= kDegH; ++k)
            s = fmaf((float)kTT.t[m][k], x[k], s);
        y[m] = s;
    }
}

__device__ __forceinline__ VoigtH voigt_setup_h(double a)
{
    // P(a - i v) = EP(u) - i v OP(u), Q(a - i v) = EQ(u) - i v OQ(u), as in
    // the FP32 setup but from the degree-4 table
    float ep[kHEP], op[kHOP], eq[kHEQ], oq[kHOQ];
#pragma unroll
    for (int m = 0; m < kHEP; ++m)
        ep[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftPH, 2 * m, a);
#pragma unroll
    for (int m = 0; m < kHOP; ++m)
        op[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftPH, 2 * m + 1, a);
#pragma unroll
    for (int m = 0; m < kHEQ; ++m)
        eq[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftQH, 2 * m, a);
#pragma unroll
    for (int m = 0; m < kHOQ; ++m)
        oq[m] = ((m & 1) ? -1.0f : 1.0f) * shifted(kShiftQH, 2 * m + 1, a);
    float nh[kNH] = {}, nl[kNH] = {}, d[kNH] = {};
    // NH = EP EQ + u OP OQ, NL = EP OQ - OP EQ, D = EQ^2 + u OQ^2
#pragma unroll
    for (int i = 0; i < kHEP; ++i) {
#pragma unroll
        for (int j = 0; j < kHEQ; ++j)
            nh[i + j] = fmaf(ep[i], eq[j], nh[i + j]);
#pragma unroll
        for (int j = 0; j < kHOQ; ++j)
            nl[i + j] = fmaf(ep[i], oq[j], nl[i + j]);
    }
#pragma unroll
    for (int i = 0; i < kHOP; ++i) {
#pragma unroll
        for (int j = 0; j < kHOQ; ++j)
            nh[i + j + 1] = fmaf(op[i], oq[j], nh[i + j + 1]);
#pragma unroll
        for (int j = 0; j < kHEQ; ++j)
            nl[i + j] = fmaf(-op[i], eq[j], nl[i + j]);
    }
#pragma unroll
    for (int i = 0; i < kHEQ; ++i)
#pragma unroll
        for (int j = 0; j < kHEQ; ++j)
            d[i + j] = fmaf(eq[i], eq[j], d[i + j]);
#pragma unroll
    for (int i = 0; i < kHOQ; ++i)
#pragma unroll
        for (int j = 0; j < kHOQ; ++j)
            d[i + j + 1] = fmaf(oq[i], oq[j], d[i + j + 1]);
    float th[kNH], tl[kNH], td[kNH];
    to_t(nh, th);
    to_t(nl, tl);
    to_t(d, td);
    float d1 = 0.0f;
#pragma unroll
    for (int m = 0; m <= kDegH; ++m)
        d1 += td[m];
    const float k = rsqrtf(td[0] * d1);
    half_t q[3 * kNH + 1];
#pragma unroll
    for (int m = 0; m <= kDegH; ++m) {
        q[m] = (half_t)(th[m] * k);
        q[kNH + m] = (half_t)(tl[m] * k);
        q[2 * kNH + m] = (half_t)(td[m] * k);
    }
    q[3 * kNH] = (half_t)0;
    VoigtH c;
#pragma unroll
    for (int i = 0; i < (3 * kNH + 1) / 2; ++i)
        c.c[i] = h2{q[2 * i], q[2 * i + 1]};
    return c;
}

__device__ __forceinline__ h2 hcoef(const VoigtH &c, int q)
{
    const half_t x = c.c[q >> 1][q & 1];
    return h2{x, x};
}

__device__ __forceinline__ h2 hfma(h2 a, h2 b, h2 c) { return __builtin_elementwise_fma(a, b, c); }

__device__ __forceinline__ h2 hrcp(h2 x)
{
    return h2{(half_t)__builtin_amdgcn_rcph(x.x), (half_t)__builtin_amdgcn_rcph(x.y)};
}

// h += w H(v), l += w L(v) for the two wavelengths of the pair.
__device__ __forceinline__ void voigt_acc_h(const VoigtH &c, h2 v, h2 w, h2 &h, h2 &l)
{
    const h2 u = v * v;
    const h2 t = hrcp(hfma(u, h2{(half_t)(1.0 / kHalfS), (half_t)(1.0 / kHalfS)},
                           h2{(half_t)1, (half_t)1}));
    h2 ph = hcoef(c, kDegH), pl = hcoef(c, kNH + kDegH), pd = hcoef(c, 2 * kNH + kDegH);
#pragma unroll
    for (int m = kDegH - 1; m >= 0; --m) {
        ph = hfma(ph, t, hcoef(c, m));
        pl = hfma(pl, t, hcoef(c, kNH + m));
        pd = hfma(pd, t, hcoef(c, 2 * kNH + m));
    }
    const h2 wr = hrcp(pd) * w;
    h = hfma(ph, wr, h);
    l = hfma(pl * v, wr, l);
}

// FP32 model constants of one individual with FP16 profile coefficients.
struct ModelH {
    float B, inv_dop, vlos;
    float cI1, cI2, cQ, cU, cV, c2;
    float S0, muS1;
    VoigtH vh;
};

__device__ __forceinline__ void model_setup(const double (&p)[GENESIS_NPAR], double mu,
                                            ModelH &m)
{
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
    m.vh = voigt_setup_h(p[5]);
}

// Component strengths of every line in FP16 (kernel argument; the shifts
// stay FP32 because the reduced wavelength is formed in FP32).
struct DevLinesH {
    half_t w[GENESIS_MAX_LINES][GENESIS_MAX_COMP];
};

template <int N>
__device__ __forceinline__ void group_h(const ModelH &m, const DevLine<float> &ln,
                                        const half_t *wh, int c0, int n, float xa, float xb,
                                        float zb, h2 &h, h2 &l)
{
    auto one = [&](int c) {
        const float s = ln.s[c];
        const h2 v = h2{(half_t)fmaf(-s, zb, xa), (half_t)fmaf(-s, zb, xb)};
        voigt_acc_h(m.vh, v, h2{wh[c], wh[c]}, h, l);
    };
    if constexpr (N >= 0) {
#pragma unroll
        for (int c = 0; c < N; ++c)
            one(c0 + c);
    } else {
        for (int c = c0; c < c0 + n; ++c)
            one(c);
    }
}

// One line, two wavelengths per iteration (the last one alone when nlam is odd).
template <int NB, int NP, int NR, typename Sink>
__device__ __forceinline__ void synth_line_h(const ModelH &m, const DevLine<float> &ln,
                                             const half_t *wh, Sink &sink)
{
    const float xb = (ln.off0 - m.vlos * ln.dop_kms) * m.inv_dop;
    const float xs = ln.step * m.inv_dop;
    const float zb = ln.zee_G * m.B * m.inv_dop;
    const int nb = NB >= 0 ? NB : ln.nb, np = NP >= 0 ? NP : ln.np;
    const int nr = NR >= 0 ? NR : ln.nr;
    for (int j = 0; j < ln.nlam; j += 2) {
        const float x0 = fmaf((float)j, xs, xb), x1 = fmaf((float)(j + 1), xs, xb);
        const h2 z = h2{(half_t)0, (half_t)0};
        h2 hb = z, lb = z, hp = z, lp = z, hr = z, lr = z;
        group_h<NB>(m, ln, wh, 0, nb, x0, x1, zb, hb, lb);
        group_h<NP>(m, ln, wh, nb, np, x0, x1, zb, hp, lp);
        group_h<NR>(m, ln, wh, nb + np, nr, x0, x1, zb, hr, lr);
        float I, Q, U, V;
        unno_rachkovsky<float>(m, (float)hb.x, (float)lb.x, (float)hp.x, (float)lp.x,
                               (float)hr.x, (float)lr.x, I, Q, U, V);
        sink(ln.off + j, I, Q, U, V);
        if (j + 1 < ln.nlam) {
            unno_rachkovsky<float>(m, (float)hb.y, (float)lb.y, (float)hp.y, (float)lp.y,
                                   (float)hr.y, (float)lr.y, I, Q, U, V);
            sink(ln.off + j + 1, I, Q, U, V);
        }
    }
}

// One line, with compile-time component counts for the two patterns of the
// Fe I pair.
template <typename Sink>
__device__ __forceinline__ void synth_line_range_h(const ModelH &m, const DevLine<float> &ln,
                                                   const half_t *wh, Sink &sink)
{
    if (ln.nb == 1 && ln.np == 1 && ln.nr == 1)
        synth_line_h<1, 1, 1>(m, ln, wh, sink);
    else if (ln.nb == 4 && ln.np == 4 && ln.nr == 4)
        synth_line_h<4, 4, 4>(m, ln, wh, sink);
    else
        synth_line_h<-1, -1, -1>(m, ln, wh, sink);
}

template <typename Sink>
__device__ __forceinline__ void synthesize_h(const ModelH &m, const DevLines<float> &ls,
                                             const DevLinesH &lh, Sink &sink)
{
    for (int l = 0; l < ls.nlines; ++l)
        synth_line_range_h(m, ls.l[l], lh.w[l], sink);
}

__device__ __forceinline__ float chi2_of_h(const ModelH &m, const DevLines<float> &ls,
                                           const DevLinesH &lh, const Vec4<float> *obs_lds,
                                           const float (&w2)[4], float inv_nu)
{
    Chi2Sink<float> s{obs_lds, 0, 0, 0, 0};
    synthesize_h(m, ls, lh, s);
    return fmaf(w2[0], s.sI, fmaf(w2[1], s.sQ, fmaf(w2[2], s.sU, w2[3] * s.sV))) * inv_nu;
}

}  // namespace genesis
