// Internal pieces shared by the translation units of libgenesis_hip.so:
// argument validation and packing on the host, and the device building
// blocks of the workgroup-per-pixel genetic-algorithm kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

#include "genesis_device.h"
#include "genesis_half.h"

namespace genesis {

// ---- host side ----------------------------------------------------------

// Record the message of a failure on this thread and return `code`.
int fail(int code, const char *fmt, ...);
// ME_EHIP with the runtime's message if the last launch failed.
int check_launch(const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kMaxGrid = 1 << 30;
constexpr size_t kMaxLds = 64 * 1024;

inline int grid_for(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>(n, 1), kMaxGrid); }
inline int block_for_pop(int pop) { return ((pop + 63) / 64) * 64; }

int pack_bounds(const me_bounds *b, Bounds &out);
int pack_ga(const ga_config *cfg, GaConst &ga);

template <typename Real>
inline int pack_lines(const me_line *lines, const me_grid *grids, int nlines, DevLines<Real> &out)
{
    if (!lines || !grids)
        return fail(ME_EINVAL, "lines and grids must not be NULL");
    if (nlines < 1 || nlines > GENESIS_MAX_LINES)
        return fail(ME_EINVAL, "nlines = %d outside [1, %d]", nlines, GENESIS_MAX_LINES);
    std::memset(&out, 0, sizeof out);
    out.nlines = nlines;
    int off = 0;
    for (int l = 0; l < nlines; ++l) {
        const me_line &ln = lines[l];
        const me_grid &gd = grids[l];
        if (!(ln.lambda0_A > 0) || !std::isfinite(ln.lambda0_A))
            return fail(ME_EINVAL, "line %d: lambda0 must be positive", l);
        if (ln.ncomp < 1 || ln.ncomp > GENESIS_MAX_COMP)
            return fail(ME_EINVAL, "line %d: ncomp = %d outside [1, %d]", l, ln.ncomp,
                        GENESIS_MAX_COMP);
        if (gd.n < 1 || !std::isfinite(gd.start_A) || !std::isfinite(gd.step_A))
            return fail(ME_EINVAL, "line %d: invalid wavelength grid", l);
        DevLine<Real> &d = out.l[l];
        d.off0 = (Real)(gd.start_A - ln.lambda0_A);
        d.step = (Real)gd.step_A;
        d.dop_kms = (Real)(ln.lambda0_A / kCkms);
        d.zee_G = (Real)(kZeeman * ln.lambda0_A * ln.lambda0_A);
        d.nlam = gd.n;
        d.off = off;
        int n = 0;
        int cnt[3] = {0, 0, 0};
        for (int g = -1; g <= 1; ++g)
            for (int c = 0; c < ln.ncomp; ++c) {
                if (ln.q[c] < -1 || ln.q[c] > 1)
                    return fail(ME_EINVAL, "line %d component %d: q must be -1, 0 or 1", l, c);
                if (!std::isfinite(ln.shift[c]) || !std::isfinite(ln.strength[c]))
                    return fail(ME_EINVAL, "line %d component %d: non-finite data", l, c);
                if (ln.q[c] != g)
                    continue;
                d.s[n] = (Real)ln.shift[c];
                d.w[n] = (Real)ln.strength[c];
                ++n;
                ++cnt[g + 1];
            }
        d.nb = cnt[0];
        d.np = cnt[1];
        d.nr = cnt[2];
        off += gd.n;
        if (off > (1 << 20))
            return fail(ME_EINVAL, "too many wavelength samples");
    }
    out.L = off;
    return ME_OK;
}

// ---- device side --------------------------------------------------------

// Code placement.  On gfx950 the profile loops of the GA kernels run about
// 20 % faster when most of their 8-byte (VOP3) instructions start at an
// address = 4 (mod 8) than when they start at 0 (mod 8) (a sweep of 0..15
// s_nop words at the entry of k_ga_invert<float>: 74.5 ms for every odd
// count, 93.4 ms for every even one, same instructions).  One s_nop at a
// kernel's entry moves all of its code by 4 bytes; the build measures the
// placement of each hot kernel's innermost loops in the compiled code object
// and sets the GENESIS_PAD_* switch of the kernels that need the shift.
#ifndef GENESIS_PAD_INVERT_F32
#define GENESIS_PAD_INVERT_F32 0
#endif
#ifndef GENESIS_PAD_INVERT_F16
#define GENESIS_PAD_INVERT_F16 0
#endif
#ifndef GENESIS_PAD_INVERT_F64
#define GENESIS_PAD_INVERT_F64 0
#endif
#ifndef GENESIS_PAD_FILL_F16
#define GENESIS_PAD_FILL_F16 0
#endif
#ifndef GENESIS_PAD_FILL_F32
#define GENESIS_PAD_FILL_F32 0
#endif
#ifndef GENESIS_PAD_FILL_F64
#define GENESIS_PAD_FILL_F64 0
#endif
#ifndef GENESIS_PAD_ADVANCE
#define GENESIS_PAD_ADVANCE 0
#endif
#ifndef GENESIS_PAD_REFINE
#define GENESIS_PAD_REFINE 0
#endif

template <int N>
__device__ __forceinline__ void code_shift()
{
    if constexpr (N > 0)
        asm volatile("s_nop 0");
}

// Stage one pixel's observation into LDS as [L] x (I, Q, U, V) and return
// its status (0 ok, 1 non-finite observation, 2 bad sigma); w2 = 1/sigma^2.
template <typename Real>
__device__ __forceinline__ int stage_pixel(const Real *__restrict__ obs_p,
                                           const Real *__restrict__ sig_p, int L,
                                           Vec4<Real> *obs_s, Real (&w2)[4])
{
    int bad = 0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        Vec4<Real> o;
        o.x = obs_p[j];
        o.y = obs_p[L + j];
        o.z = obs_p[2 * L + j];
        o.w = obs_p[3 * L + j];
        bad |= !(isfinite(o.x) && isfinite(o.y) && isfinite(o.z) && isfinite(o.w));
        obs_s[j] = o;
    }
    bad = __syncthreads_or(bad);
    int bad_sig = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const Real sg = sig_p[s];
        bad_sig |= !(sg > (Real)0 && isfinite(sg));
        w2[s] = (Real)1 / (sg * sg);
    }
    return bad ? 1 : (bad_sig ? 2 : 0);
}

// ---- magnetic fill fraction (Sec. 5.2) --------------------------------------
// A fraction alpha of the pixel is magnetic, the rest field-free:
//   alpha M(p) + (1 - alpha) I_c N(lambda) e,   I_c = S0 + mu S1,
// N = 1 - d(mu) H(v, a(mu)) / H(0, a(mu)), v = (lambda - lambda0 (1 + v_los/c))
// / w(mu), with depth d, width w and damping a cubic polynomials in mu (inputs:
// the paper's centre-to-limb fits are not published).  alpha enters linearly,
// so each model takes its chi-square-optimal alpha in [alpha_lo, alpha_hi] in
// closed form; with e = O - M (the residual at alpha = 1) and D = M - I_c N e,
//   chi2(beta) nu = sum w^2 e.e + 2 beta sum w^2 e.D + beta^2 sum w^2 D.D,
// beta = 1 - alpha, minimised at beta = -sum w^2 e.D / sum w^2 D.D (clamped;
// alpha_hi where sum w^2 D.D = 0); nu = 4L - 10.

struct FillConst {
    double alpha_lo, alpha_hi;
    double depth[GENESIS_MAX_LINES][4], width[GENESIS_MAX_LINES][4], damp[GENESIS_MAX_LINES][4];
};

// The fill-fraction constants of a me_fill (host; checks the alpha range and
// that the coefficients of the first nlines lines are finite).
int pack_fill(const me_fill *fill, int nlines, FillConst &fc);

template <typename Real>
struct FillLine;
template <>
struct FillLine<float> {
    VoigtF32 vc;            // rational-approximation coefficients at a(mu)
    float scale, inv_w, a;  // d / H(0, a), 1 / w, a
};
template <>
struct FillLine<double> {
    double a, scale, inv_w;
};

template <typename Real>
struct FillPix {
    FillLine<Real> l[GENESIS_MAX_LINES];
    int status;  // 0, or 4 when the field-free profile is invalid at this mu
};

__device__ __forceinline__ double cubic_mu(const double (&c)[4], double mu)
{
    return c[0] + mu * (c[1] + mu * (c[2] + mu * c[3]));
}

// The field-free profile constants of line l at this mu; false when the
// width is not positive or the damping outside [0, 1.5].
template <typename Real>
__device__ __forceinline__ bool fill_setup_line(const FillConst &fc, int l, double mu,
                                                FillLine<Real> &f)
{
    const double d = cubic_mu(fc.depth[l], mu), w = cubic_mu(fc.width[l], mu),
                 a = cubic_mu(fc.damp[l], mu);
    if (!(isfinite(d) && isfinite(w) && isfinite(a) && w > 0.0 && a >= 0.0 && a <= 1.5))
        return false;
    if constexpr (std::is_same<Real, float>::value) {
        f.vc = voigt_setup_f32(a);
        f.a = (float)a;
        float h0 = 0.0f, l0 = 0.0f;
        voigt_acc_f32(f.vc, 0.0f, 1.0f, h0, l0);
        f.scale = (float)d / h0;
    } else {
        double h0, l0;
        voigt_f64(a, 0.0, h0, l0);
        f.a = a;
        f.scale = d / h0;
    }
    f.inv_w = (Real)(1.0 / w);
    return true;
}

// ... of every line (one thread).
template <typename Real>
__device__ __forceinline__ void fill_setup(const FillConst &fc, int nlines, double mu,
                                           FillPix<Real> &fp)
{
    fp.status = 0;
    for (int l = 0; l < nlines; ++l)
        if (!fill_setup_line(fc, l, mu, fp.l[l])) {
            fp.status = 4;
            return;
        }
}

__device__ __forceinline__ float fill_h(const FillLine<float> &f, float v)
{
    // The rational's |Q|^2 grows like v^16 and overflows FP32 from |v| ~ 250,
    // which a field-free width near zero reaches (the magnetic profiles stay
    // below |v| ~ 50).  Beyond |v| = 100 the Lorentzian wing a / (sqrt(pi)
    // (v^2 + a^2)) is good to ~1e-4 relative, ~1e-9 absolute.
    if (fabsf(v) > 100.0f)
        return f.a * 0.5641895835f / fmaf(v, v, f.a * f.a);
    float h = 0.0f, l = 0.0f;
    voigt_acc_f32(f.vc, v, 1.0f, h, l);
    return h;
}

__device__ __forceinline__ double fill_h(const FillLine<double> &f, double v)
{
    double h, l;
    voigt_f64(f.a, v, h, l);
    return h;
}

// Accumulates sum w^2 e.e, e.D and D.D of one model against the staged
// observation while the Stokes vector is synthesised.
template <typename Real>
struct FillSink {
    const Vec4<Real> *obs;
    const FillLine<Real> *fl;
    const DevLine<Real> *ln;
    Real vshift, ic;
    Real w2[4];
    Real see, sed, sdd;
    __device__ __forceinline__ void operator()(int j, Real I, Real Q, Real U, Real V)
    {
        const Real x = fma(ln->step, (Real)(j - ln->off), ln->off0);
        const Real N = fma(-fl->scale, fill_h(*fl, (x - vshift) * fl->inv_w), (Real)1);
        const Real dI = fma(-ic, N, I);  // D_I = I - I_c N; D_Q,U,V = Q, U, V
        const Vec4<Real> o = obs[j];
        const Real eI = o.x - I, eQ = o.y - Q, eU = o.z - U, eV = o.w - V;
        const Real wI = w2[0] * eI, wQ = w2[1] * eQ, wU = w2[2] * eU, wV = w2[3] * eV;
        see = fma(wI, eI, fma(wQ, eQ, fma(wU, eU, fma(wV, eV, see))));
        sed = fma(wI, dI, fma(wQ, Q, fma(wU, U, fma(wV, V, sed))));
        sdd = fma(w2[0] * dI, dI, fma(w2[1] * Q, Q, fma(w2[2] * U, U, fma(w2[3] * V, V, sdd))));
    }
};

template <typename Real, typename M>
__device__ __forceinline__ FillSink<Real> fill_sink(const M &m, const Vec4<Real> *obs_s,
                                                    const Real (&w2)[4])
{
    FillSink<Real> s;
    s.obs = obs_s;
    s.ic = m.S0 + m.muS1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        s.w2[k] = w2[k];
    s.see = s.sed = s.sdd = (Real)0;
    return s;
}

// The chi-square's minimum over alpha in [alo, ahi] from the sums, and that alpha.
template <typename Real>
__device__ __forceinline__ Real fill_minimum(const FillSink<Real> &s, Real alo, Real ahi,
                                             Real inv_nu, Real &alpha)
{
    const Real bmin = (Real)1 - ahi, bmax = (Real)1 - alo;
    Real beta = s.sdd > (Real)0 ? -s.sed / s.sdd : bmin;
    beta = fmin(fmax(beta, bmin), bmax);
    alpha = (Real)1 - beta;
    return fma(beta, fma(beta, s.sdd, (Real)2 * s.sed), s.see) * inv_nu;
}

// chi-square at the model's best fill fraction, and that fraction.
template <typename Real>
__device__ __forceinline__ Real chi2_fill_of(const Model<Real> &m, const DevLines<Real> &ls,
                                             const FillPix<Real> &fp, Real alo, Real ahi,
                                             const Vec4<Real> *obs_s, const Real (&w2)[4],
                                             Real inv_nu, Real &alpha)
{
    FillSink<Real> s = fill_sink<Real>(m, obs_s, w2);
    for (int l = 0; l < ls.nlines; ++l) {
        const DevLine<Real> &ln = ls.l[l];
        s.ln = &ln;
        s.fl = &fp.l[l];
        s.vshift = m.vlos * ln.dop_kms;
        synth_line_range(m, ln, s, 0, ln.nlam);
    }
    return fill_minimum(s, alo, ahi, inv_nu, alpha);
}

// The same with the magnetic profiles synthesised in packed FP16 (the
// field-free profile, the mixture and the sums in FP32).
__device__ __forceinline__ float chi2_fill_of_h(const ModelH &m, const DevLines<float> &ls,
                                                const DevLinesH &lh, const FillPix<float> &fp,
                                                float alo, float ahi, const Vec4<float> *obs_s,
                                                const float (&w2)[4], float inv_nu, float &alpha)
{
    FillSink<float> s = fill_sink<float>(m, obs_s, w2);
    for (int l = 0; l < ls.nlines; ++l) {
        const DevLine<float> &ln = ls.l[l];
        s.ln = &ln;
        s.fl = &fp.l[l];
        s.vshift = m.vlos * ln.dop_kms;
        synth_line_range_h(m, ln, lh.w[l], s);
    }
    return fill_minimum(s, alo, ahi, inv_nu, alpha);
}

// LDS of the GA kernels: observation [L] x 4, fitness [pop], argmin
// scratch, two gene buffers [9][pop] (parents, children) and the pixel's
// search box.
template <typename Real>
struct GaLds {
    Vec4<Real> *obs;
    Real *fit, *red_f;
    int *red_i;
    unsigned long long *tick;  // the progress count seen by this workgroup (see generation_loop)
    uint16_t *genes;  // two buffers [9][pop] back to back
    Bounds *box;
    void *fill;       // FillPix<Real> of the pixel (fill-fraction kernels)
};

// The search box of pixel p, written by one thread: its row of
// pixel_bounds [npix][2][9] (lo, hi) when given, else the common box.
__device__ __forceinline__ void stage_box(const Bounds &common, const float *pixel_bounds,
                                          int64_t p, Bounds &box)
{
    if (!pixel_bounds) {
#pragma unroll
        for (int j = 0; j < GENESIS_NPAR; ++j) {
            box.lo[j] = common.lo[j];
            box.span[j] = common.span[j];
        }
        return;
    }
    const float *row = pixel_bounds + p * 2 * GENESIS_NPAR;
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        const double lo = (double)row[j], hi = (double)row[GENESIS_NPAR + j];
        box.lo[j] = lo;
        box.span[j] = hi - lo;  // exact for two floats
    }
}

// 0, or 3 for a box that is not finite with hi >= lo or, for the FP16
// synthesis, has damping outside [0, 1].
__device__ __forceinline__ int box_status(const Bounds &box, bool fp16)
{
    for (int j = 0; j < GENESIS_NPAR; ++j)
        if (!(isfinite(box.lo[j]) && isfinite(box.span[j]) && box.span[j] >= 0.0))
            return 3;
    if (fp16 && !(box.lo[5] >= 0.0 && box.lo[5] + box.span[5] <= 1.0))
        return 3;
    return 0;
}

__host__ __device__ inline size_t align16(size_t o) { return (o + 15) & ~(size_t)15; }

template <typename Real>
__host__ __device__ inline size_t ga_lds_bytes(int L, int pop)
{
    size_t o = align16(sizeof(Vec4<Real>) * (size_t)L);
    o = align16(o + sizeof(Real) * (size_t)pop);
    o += (sizeof(Real) + sizeof(int)) * 16 + 16;
    o = align16(o + 2 * sizeof(uint16_t) * GENESIS_NPAR * (size_t)pop);
    o = align16(o + sizeof(Bounds));
    o = align16(o + sizeof(FillPix<Real>));
    return o;
}

template <typename Real>
__device__ __forceinline__ GaLds<Real> ga_lds(unsigned char *base, int L, int pop)
{
    GaLds<Real> s;
    size_t o = 0;
    s.obs = reinterpret_cast<Vec4<Real> *>(base);
    o = align16(sizeof(Vec4<Real>) * (size_t)L);
    s.fit = reinterpret_cast<Real *>(base + o);
    o = align16(o + sizeof(Real) * (size_t)pop);
    s.red_f = reinterpret_cast<Real *>(base + o);
    o += sizeof(Real) * 16;
    s.red_i = reinterpret_cast<int *>(base + o);
    o += sizeof(int) * 16;
    s.tick = reinterpret_cast<unsigned long long *>(base + o);
    o += 16;
    s.genes = reinterpret_cast<uint16_t *>(base + o);
    o = align16(o + 2 * sizeof(uint16_t) * GENESIS_NPAR * (size_t)pop);
    s.box = reinterpret_cast<Bounds *>(base + o);
    o = align16(o + sizeof(Bounds));
    s.fill = base + o;
    return s;
}

// Child sink writing into an LDS gene buffer [9][pop].
struct LdsChild {
    uint16_t *dst;
    int pop, c;
    __device__ __forceinline__ void meta(int, int, int) {}
    __device__ __forceinline__ void gene(int j, uint32_t g, uint32_t)
    {
        dst[j * pop + c] = (uint16_t)g;
    }
};

template <typename Real>
__device__ __forceinline__ Real evaluate_lds(const uint16_t *genes_s, int pop, int i,
                                             const Bounds &b, double mu,
                                             const DevLines<Real> &ls, const Vec4<Real> *obs_s,
                                             const Real (&w2)[4], Real inv_nu)
{
    uint32_t g[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        g[j] = genes_s[j * pop + i];
    double par[GENESIS_NPAR];
    decode(g, b, par);
    Model<Real> m;
    model_setup(par, mu, m);
    return chi2_of(m, ls, obs_s, w2, inv_nu);
}

template <typename Real>
__device__ __forceinline__ Real evaluate_fill(const uint16_t *genes_s, int pop, int i,
                                              const Bounds &b, double mu,
                                              const DevLines<Real> &ls, const FillPix<Real> &fp,
                                              Real alo, Real ahi, const Vec4<Real> *obs_s,
                                              const Real (&w2)[4], Real inv_nu, Real &alpha)
{
    uint32_t g[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        g[j] = genes_s[j * pop + i];
    double par[GENESIS_NPAR];
    decode(g, b, par);
    Model<Real> m;
    model_setup(par, mu, m);
    return chi2_fill_of(m, ls, fp, alo, ahi, obs_s, w2, inv_nu, alpha);
}

// FP16-synthesis variant of evaluate_lds (FP32 decode set-up and chi-square).
__device__ __forceinline__ float evaluate_lds_h(const uint16_t *genes_s, int pop, int i,
                                                const Bounds &b, double mu,
                                                const DevLines<float> &ls, const DevLinesH &lh,
                                                const Vec4<float> *obs_s, const float (&w2)[4],
                                                float inv_nu)
{
    uint32_t g[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        g[j] = genes_s[j * pop + i];
    double par[GENESIS_NPAR];
    decode(g, b, par);
    ModelH m;
    model_setup(par, mu, m);
    return chi2_of_h(m, ls, lh, obs_s, w2, inv_nu);
}

// Issue priority of the calling wave, 0 (lowest) to 3; the instruction takes
// an immediate, so the four values are four branches (uniform per wave).
__device__ __forceinline__ void set_issue_priority(int r)
{
    switch (r & 3) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Where a pixel's generation loop stands: generation g with its genes at
// s.genes + cur; `eval` when this lane's individual still has to be
// evaluated, `restarted` once generation g's restart (if due) is done.
template <typename Real>
struct GenState {
    int g, cur;
    bool eval, restarted;
    Real f;  // this lane's fitness of generation g (once evaluated)
};

// The generation loop of Algorithm 1 for one pixel (one workgroup, lane i
// owns individual i; parents and children in the two LDS gene buffers):
// evaluate generation g, restart it when due (Sec. 5.6; the replaced lanes
// come back here to be evaluated), and breed generation g + 1 (elite to slot
// 0, selection, recombination, mutation), until generation g_to is evaluated
// and restarted.  evaluate(genes) returns the calling lane's fitness of the
// genes in buffer `genes`.  With a progress counter (the whole launch
// resident at once; see k_ga_invert) each workgroup raises its waves' issue
// priority while it lags the average generation of the workgroups on its XCD.
// On return s.fit holds generation g_to's fitness.  ga_invert and the
// service run this same loop, so a served pixel is bit-identical to it.
template <typename Real, typename Eval>
__device__ __forceinline__ void generation_loop(const GaLds<Real> &s, int pop, int tid,
                                                uint32_t pix, const GaConst &ga,
                                                int generations, int g_to,
                                                unsigned long long *progress,
                                                GenState<Real> &st, Eval &&evaluate)
{
    const bool active = tid < pop;
    const int gstride = GENESIS_NPAR * pop;
    for (;;) {
        // Progress: once per generation thread 0 adds to the counter (high
        // word: workgroups started, low word: generations begun) and keeps
        // the count it saw; at the next generation every wave sets its
        // priority from how far this workgroup was behind the average then.
        const bool count = progress != nullptr && !st.restarted;
        if (count && st.g > 0) {
            const unsigned long long t = *s.tick;
            const long long started = (long long)(t >> 32), begun = (long long)(t & 0xffffffffu);
            const long long d = begun - (long long)(st.g - 1) * started;
            set_issue_priority(d >= started ? 3 : (2 * d >= started ? 2 : (d >= 0 ? 1 : 0)));
        }
        unsigned long long tick = 0;
        if (count && tid == 0)
            tick = __hip_atomic_fetch_add(progress, st.g == 0 ? (1ull << 32) + 1ull : 1ull,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (st.eval) {
            st.f = evaluate(s.genes + st.cur);
            s.fit[tid] = st.f;
        }
        __syncthreads();
        if (count && tid == 0)
            *s.tick = tick;
        if (!st.restarted && restart_due(ga, st.g, generations)) {
            const int rank = active ? fitness_rank(s.fit, pop, tid) : 0;
            __syncthreads();
            uint32_t gr[GENESIS_NPAR];
            st.eval = active && restart_genes(ga, pix, st.g, rank, gr);
            if (st.eval)
#pragma unroll
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    s.genes[st.cur + j * pop + tid] = (uint16_t)gr[j];
            st.restarted = true;
            continue;
        }
        if (st.g == g_to)
            break;
        const int e = block_argmin(s.fit, pop, s.red_f, s.red_i);
        if (active) {
            LdsChild out{s.genes + (gstride - st.cur), pop, tid};
            if (tid == 0) {
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    out.gene(j, s.genes[st.cur + j * pop + e], 0u);
            } else {
                make_child(tid, pix, (uint32_t)(st.g + 1), s.fit, s.genes + st.cur, ga, out);
            }
        }
        __syncthreads();
        st.cur = gstride - st.cur;
        ++st.g;
        st.eval = active;
        st.restarted = false;
    }
}

// Generation 0 of one pixel into the first gene buffer (Algorithm 1,
// "Create P0"), to be evaluated by generation_loop.
template <typename Real>
__device__ __forceinline__ GenState<Real> generation_zero(const GaLds<Real> &s, int pop, int tid,
                                                         uint32_t pix, int64_t p,
                                                         const GaConst &ga)
{
    if (tid < pop) {
        uint32_t g0[GENESIS_NPAR];
        initial_genes(pix, p, tid, ga, *s.box, g0);
#pragma unroll
        for (int j = 0; j < GENESIS_NPAR; ++j)
            s.genes[j * pop + tid] = (uint16_t)g0[j];
    }
    return GenState<Real>{0, 0, tid < pop, false, (Real)0};
}

// The best individual of the current generation (elite rule: least fitness,
// ties to the lower index, NaN last): its decoded parameters on thread 0.
template <typename Real>
__device__ __forceinline__ int best_of(const GaLds<Real> &s, int pop, const GenState<Real> &st,
                                       double (&par)[GENESIS_NPAR])
{
    const int e = block_argmin(s.fit, pop, s.red_f, s.red_i);
    if (threadIdx.x == 0) {
        uint32_t gb[GENESIS_NPAR];
        for (int j = 0; j < GENESIS_NPAR; ++j)
            gb[j] = s.genes[st.cur + j * pop + e];
        decode(gb, *s.box, par);
    }
    return e;
}

// FP16-synthesis variant of evaluate_fill.
__device__ __forceinline__ float evaluate_fill_h(const uint16_t *genes_s, int pop, int i,
                                                 const Bounds &b, double mu,
                                                 const DevLines<float> &ls, const DevLinesH &lh,
                                                 const FillPix<float> &fp, float alo, float ahi,
                                                 const Vec4<float> *obs_s, const float (&w2)[4],
                                                 float inv_nu, float &alpha)
{
    uint32_t g[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        g[j] = genes_s[j * pop + i];
    double par[GENESIS_NPAR];
    decode(g, b, par);
    ModelH m;
    model_setup(par, mu, m);
    return chi2_fill_of_h(m, ls, lh, fp, alo, ahi, obs_s, w2, inv_nu, alpha);
}

// FP16 strength table of packed lines (after pack_lines).
inline void pack_lines_h(const DevLines<float> &ls, DevLinesH &out)
{
    std::memset(&out, 0, sizeof out);
    for (int l = 0; l < ls.nlines; ++l)
        for (int c = 0; c < GENESIS_MAX_COMP; ++c)
            out.w[l][c] = (half_t)ls.l[l].w[c];
}

}  // namespace genesis
