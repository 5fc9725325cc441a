// Uncertainties of the fitted parameters at the optimum (Sec. 6), FP64.
//
// Sec. 6 differentiates the merit function (the chi-square of Sec. 5) at the
// optimum with steps set by the spread of the final population, sharpens the
// derivatives by Richardson extrapolation to zero step in Neville's scheme,
// takes the Hessian H as the Jacobian of that gradient, and reports
// sigma_j^2 = [H^-1]_jj chi2(p_opt) / M.
//
// One derivative (Ridders' extrapolation): central differences
// D_k = (F(x + t_k) - F(x - t_k)) / (2 t_k), t_k = h / 1.4^k, k < 10, fill the
// Neville tableau T[k][0] = D_k, T[k][m] = (c T[k][m-1] - T[k-1][m-1]) / (c - 1),
// c = 1.4^2m; each entry's error is the larger difference to its parents; the
// answer is the entry of smallest error, and a component stops after the row
// whose diagonal moved by at least twice that error.  The gradient runs one
// tableau per parameter; Hessian column j runs one tableau per gradient
// component on the gradients at p +- t e_j; H is symmetrised.
//
// Layout: one workgroup per pixel, threads over wavelengths (as in the
// refinement).  Every tableau level of the gradient is one batch: the up to
// 18 stencil points of the live components are set up by 18 lanes and
// evaluated in one sweep over the wavelengths with one workgroup reduction.
// A point that differs from the gradient's base point only in the angles,
// eta0, S0 or S1 has the base point's Voigt and Faraday-Voigt profiles
// (they depend on B, v_los, the Doppler width and the damping only), so the
// sweep computes those profiles once per wavelength and only the
// Unno-Rachkovsky algebra per such point; the values are the same to the bit.
#include <hip/hip_runtime.h>

#include "genesis_common.h"
#include "weideman28.h"

using namespace genesis;

namespace {

constexpr int kUncThreads = 128;
constexpr int kSlots = 2 * GENESIS_NPAR;
constexpr int kTab = 10;
constexpr double kStepRatio = 1.4;
constexpr double kSafe = 2.0;

struct UncArgs {
    const double *obs, *sigma, *mu, *p_opt, *steps;
    int64_t npix;
    DevLines<double> ls;
    double lo[GENESIS_NPAR], hi[GENESIS_NPAR];
    uint32_t free_mask;
    int32_t M;
    double *sigma_out, *hess, *hess_err, *steps_used;
};

// Ridders tableaux of up to 9 components.
struct Tableau {
    double prev[kTab][GENESIS_NPAR], cur[kTab][GENESIS_NPAR];
    double best[GENESIS_NPAR], err[GENESIS_NPAR], t[GENESIS_NPAR];
    int live[GENESIS_NPAR];
    int nlive;
};

struct UncShared {
    Model<double> mod[kSlots];
    Model<double> base;              // the gradient's base point q
    double p[GENESIS_NPAR], h[GENESIS_NPAR], q[GENESIS_NPAR];
    int act[GENESIS_NPAR];
    int slot_of[GENESIS_NPAR];       // component -> first of its two slots
    int own[kSlots];                 // slot needs its own profiles
    int nslots, need_base;           // slots in the batch; some slot uses the base profiles
    double f[kSlots];
    double acc[kSlots][kUncThreads];
    double red[kUncThreads / 64][kSlots];
    Tableau in, out;
    double gp[GENESIS_NPAR], gm[GENESIS_NPAR];
    double H[GENESIS_NPAR][GENESIS_NPAR], He[GENESIS_NPAR][GENESIS_NPAR];
    double chi2;
    int flag;
};

// parameters whose change alters the group profiles
__device__ __forceinline__ bool moves_profiles(int i) { return i == 0 || (i >= 3 && i <= 5); }

// Start a tableau for the components in mask, initial steps h.
__device__ void tab_init(Tableau &T, const int *mask, const double *h)
{
    if (threadIdx.x == 0) {
        T.nlive = 0;
        for (int i = 0; i < GENESIS_NPAR; ++i) {
            T.live[i] = mask[i];
            T.nlive += mask[i];
            T.best[i] = NAN;
            T.err[i] = HUGE_VAL;
            T.t[i] = h[i];
        }
    }
}

// Row k of component i from its central difference d (thread i).
__device__ void tab_row(Tableau &T, int i, int k, double d)
{
    T.cur[0][i] = d;
    if (k == 0) {
        T.best[i] = d;
    } else {
        double fac = kStepRatio * kStepRatio;
        for (int m = 1; m <= k; ++m, fac *= kStepRatio * kStepRatio) {
            T.cur[m][i] = (T.cur[m - 1][i] * fac - T.prev[m - 1][i]) / (fac - 1.0);
            const double e = fmax(fabs(T.cur[m][i] - T.cur[m - 1][i]),
                                  fabs(T.cur[m][i] - T.prev[m - 1][i]));
            if (e <= T.err[i]) {
                T.err[i] = e;
                T.best[i] = T.cur[m][i];
            }
        }
        if (fabs(T.cur[k][i] - T.prev[k - 1][i]) >= kSafe * T.err[i])
            T.live[i] = 0;
    }
    for (int m = 0; m <= k; ++m)
        T.prev[m][i] = T.cur[m][i];
}

__device__ void tab_count(Tableau &T)
{
    if (threadIdx.x == 0) {
        int n = 0;
        for (int i = 0; i < GENESIS_NPAR; ++i)
            n += T.live[i];
        T.nlive = n;
    }
}

// Components of one Zeeman group (as group() in genesis_device.h), each
// profile from Weideman's expansion at N = 28: error about 2e-12 against
// 2e-15 at the FP64 kernels' N = 36, smooth in z (the difference of two
// analytic functions), far below what the central differences resolve, and
// 22 % fewer operations per component.
template <int N>
__device__ __forceinline__ void group28(const Model<double> &m, const DevLine<double> &ln, int c0,
                                        int n, double x0, double zb, double &h, double &l)
{
    auto acc = [&](int c) {
        double H, L;
        weideman_w(genesis_wd28_c, GENESIS_WD28_L, m.a, fma(-ln.s[c], zb, x0), H, L);
        h = fma(ln.w[c], H, h);
        l = fma(ln.w[c], L, l);
    };
    if constexpr (N >= 0) {
#pragma unroll
        for (int c = 0; c < N; ++c)
            acc(c0 + c);
    } else {
        for (int c = c0; c < c0 + n; ++c)
            acc(c);
    }
}

// The three group profiles at sample jj with compile-time component counts
// where the line has them (the components' Faddeeva evaluations are then
// independent chains the scheduler can interleave); N = 36 (the FP64 forward
// model's) if W36, else N = 28.
template <int NB, int NP, int NR, bool W36>
__device__ __forceinline__ void profiles_n(const Model<double> &m, const DevLine<double> &ln,
                                           int jj, double (&pr)[6])
{
    const double xb = (ln.off0 - m.vlos * ln.dop_kms) * m.inv_dop;
    const double x0 = fma((double)jj, ln.step * m.inv_dop, xb);
    const double zb = ln.zee_G * m.B * m.inv_dop;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        pr[i] = 0.0;
    if constexpr (W36) {
        group<NB>(m, ln, 0, ln.nb, x0, zb, pr[0], pr[1]);
        group<NP>(m, ln, ln.nb, ln.np, x0, zb, pr[2], pr[3]);
        group<NR>(m, ln, ln.nb + ln.np, ln.nr, x0, zb, pr[4], pr[5]);
    } else {
        group28<NB>(m, ln, 0, ln.nb, x0, zb, pr[0], pr[1]);
        group28<NP>(m, ln, ln.nb, ln.np, x0, zb, pr[2], pr[3]);
        group28<NR>(m, ln, ln.nb + ln.np, ln.nr, x0, zb, pr[4], pr[5]);
    }
}

// One sample of one line for every slot of the batch.  Slots come in pairs
// (q + t e_i, q - t e_i) that both need their own profiles or both take the
// base point's; a pair's two evaluations sit in one block so that they
// interleave.  A batch of one slot (chi2 at the optimum) evaluates it twice.
template <int NB, int NP, int NR, bool W36>
__device__ __forceinline__ void sweep_sample(UncShared &sh, const DevLine<double> &ln, int jj,
                                             const Vec4<double> &o, const double (&w2)[4],
                                             int ns, int tid)
{
    double pr0[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (sh.need_base)
        profiles_n<NB, NP, NR, W36>(sh.base, ln, jj, pr0);
    for (int s = 0; s < ns; s += 2) {
        const int s1 = s + 1 < ns ? s + 1 : s;
        double S[2][4];
        if (sh.own[s]) {
            double pa[6], pb[6];
            profiles_n<NB, NP, NR, W36>(sh.mod[s], ln, jj, pa);
            profiles_n<NB, NP, NR, W36>(sh.mod[s1], ln, jj, pb);
            unno_rachkovsky(sh.mod[s], pa[0], pa[1], pa[2], pa[3], pa[4], pa[5], S[0][0],
                            S[0][1], S[0][2], S[0][3]);
            unno_rachkovsky(sh.mod[s1], pb[0], pb[1], pb[2], pb[3], pb[4], pb[5], S[1][0],
                            S[1][1], S[1][2], S[1][3]);
        } else {
            unno_rachkovsky(sh.mod[s], pr0[0], pr0[1], pr0[2], pr0[3], pr0[4], pr0[5], S[0][0],
                            S[0][1], S[0][2], S[0][3]);
            unno_rachkovsky(sh.mod[s1], pr0[0], pr0[1], pr0[2], pr0[3], pr0[4], pr0[5],
                            S[1][0], S[1][1], S[1][2], S[1][3]);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double dI = o.x - S[k][0], dQ = o.y - S[k][1], dU = o.z - S[k][2],
                         dV = o.w - S[k][3];
            const double r =
                w2[0] * dI * dI + w2[1] * dQ * dQ + w2[2] * dU * dU + w2[3] * dV * dV;
            if (k == 0 || s1 != s)
                sh.acc[s + k][tid] += r;
        }
    }
}

// chi2 (reduced) of the batch's slots into sh.f.  Each thread accumulates
// its wavelengths' squared residuals per slot in its own LDS column; it reads
// its samples of the observation obs_p [4][L] from memory (cached: the batch
// count keeps them hot), so the observation's length is not bounded by LDS.
// W36:
// profiles with the forward model's N = 36 (the chi-square at the optimum, so
// that it is the one the search and the refinement minimise).
template <bool W36>
__device__ __forceinline__ void eval_batch(const UncArgs &a, UncShared &sh,
                                           const double *__restrict__ obs_p,
                                           const double (&w2)[4], double inv_nu)
{
    const int ns = sh.nslots;
    const int tid = threadIdx.x;
    for (int s = 0; s < ns; ++s)
        sh.acc[s][tid] = 0.0;
    for (int l = 0; l < a.ls.nlines; ++l) {
        const DevLine<double> &ln = a.ls.l[l];
        for (int jj = tid; jj < ln.nlam; jj += kUncThreads) {
            const int j = ln.off + jj, L = a.ls.L;
            const Vec4<double> o{obs_p[j], obs_p[L + j], obs_p[2 * L + j], obs_p[3 * L + j]};
            if (ln.nb == 1 && ln.np == 1 && ln.nr == 1)
                sweep_sample<1, 1, 1, W36>(sh, ln, jj, o, w2, ns, tid);
            else if (ln.nb == 4 && ln.np == 4 && ln.nr == 4)
                sweep_sample<4, 4, 4, W36>(sh, ln, jj, o, w2, ns, tid);
            else
                sweep_sample<-1, -1, -1, W36>(sh, ln, jj, o, w2, ns, tid);
        }
    }
    const int w = tid >> 6;
    for (int s = 0; s < ns; ++s) {
        double v = sh.acc[s][tid];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            v += __shfl_xor(v, off);
        if ((tid & 63) == 0)
            sh.red[w][s] = v;
    }
    __syncthreads();
    if (tid < ns) {
        double t = 0.0;
        for (int k = 0; k < kUncThreads / 64; ++k)
            t += sh.red[k][tid];
        sh.f[tid] = t * inv_nu;
    }
    __syncthreads();
}

// Gradient at sh.q for the components in mask (LDS) into g (LDS).
__device__ void gradient(const UncArgs &a, UncShared &sh, const int *mask, double *g,
                         double mu, const double *__restrict__ obs_p, const double (&w2)[4],
                         double inv_nu)
{
    const int tid = threadIdx.x;
    tab_init(sh.in, mask, sh.h);
    if (tid == GENESIS_NPAR) {
        double q[GENESIS_NPAR];
        for (int j = 0; j < GENESIS_NPAR; ++j)
            q[j] = sh.q[j];
        model_setup(q, mu, sh.base);
    }
    __syncthreads();
    for (int k = 0; k < kTab && sh.in.nlive > 0; ++k) {
        if (tid == 0) {
            int n = 0, nb = 0;
            for (int i = 0; i < GENESIS_NPAR; ++i)
                if (sh.in.live[i]) {
                    sh.slot_of[i] = n;
                    sh.own[n] = sh.own[n + 1] = moves_profiles(i) ? 1 : 0;
                    nb += moves_profiles(i) ? 0 : 1;
                    n += 2;
                }
            sh.nslots = n;
            sh.need_base = nb > 0;
        }
        __syncthreads();
        if (tid < sh.nslots) {
            // slot 2m: q + t e_i, slot 2m + 1: q - t e_i for the m-th live i
            int i = -1;
            for (int c = 0; c < GENESIS_NPAR; ++c)
                if (sh.in.live[c] && sh.slot_of[c] == (tid & ~1))
                    i = c;
            double x[GENESIS_NPAR];
            for (int j = 0; j < GENESIS_NPAR; ++j)
                x[j] = sh.q[j];
            if (i >= 0) {
                if (tid & 1)
                    x[i] -= sh.in.t[i];
                else
                    x[i] += sh.in.t[i];
            }
            model_setup(x, mu, sh.mod[tid]);
        }
        __syncthreads();
        eval_batch<false>(a, sh, obs_p, w2, inv_nu);
        if (tid < GENESIS_NPAR && sh.in.live[tid]) {
            const int s = sh.slot_of[tid];
            const double t = sh.in.t[tid];
            tab_row(sh.in, tid, k, (sh.f[s] - sh.f[s + 1]) / (2.0 * t));
            sh.in.t[tid] = t / kStepRatio;
        }
        __syncthreads();
        tab_count(sh.in);
        __syncthreads();
    }
    if (tid < GENESIS_NPAR)
        g[tid] = mask[tid] ? sh.in.best[tid] : 0.0;
    __syncthreads();
}

// sigma_j^2 = [H^-1]_jj c / M over the active parameters with H_jj != 0
// (NaN inactive, +inf where H_jj = 0, NaN everywhere when the kept block is
// not positive definite).  Thread 0.
__device__ void sigmas(const UncShared &sh, double c, int M, double *out)
{
    int keep[GENESIS_NPAR], idx[GENESIS_NPAR], m = 0;
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        keep[j] = sh.act[j] && sh.H[j][j] != 0.0;
        out[j] = !sh.act[j] ? NAN : (keep[j] ? 0.0 : INFINITY);
        if (keep[j])
            idx[m++] = j;
    }
    if (m == 0)
        return;
    double Lm[GENESIS_NPAR][GENESIS_NPAR];
    for (int r = 0; r < m; ++r)
        for (int s = 0; s <= r; ++s) {
            double v = sh.H[idx[r]][idx[s]];
            for (int k = 0; k < s; ++k)
                v -= Lm[r][k] * Lm[s][k];
            if (r == s) {
                if (!(v > 0.0)) {
                    for (int j = 0; j < GENESIS_NPAR; ++j)
                        out[j] = NAN;
                    return;
                }
                Lm[r][r] = sqrt(v);
            } else {
                Lm[r][s] = v / Lm[s][s];
            }
        }
    for (int r = 0; r < m; ++r) {
        double y[GENESIS_NPAR], z[GENESIS_NPAR];
        for (int u = 0; u < m; ++u) {
            double v = u == r ? 1.0 : 0.0;
            for (int k = 0; k < u; ++k)
                v -= Lm[u][k] * z[k];
            z[u] = v / Lm[u][u];
        }
        for (int u = m - 1; u >= 0; --u) {
            double v = z[u];
            for (int k = u + 1; k < m; ++k)
                v -= Lm[k][u] * y[k];
            y[u] = v / Lm[u][u];
        }
        out[idx[r]] = sqrt(y[r] * c / (double)M);
    }
}

// Status of a pixel's inputs (0 ok, 1 non-finite observation, 2 sigma <= 0
// or non-finite) and its weights w2 = 1/sigma^2.
__device__ __forceinline__ int check_pixel(const double *__restrict__ obs_p,
                                           const double *__restrict__ sig_p, int L,
                                           double (&w2)[4])
{
    int bad = 0;
    for (int j = threadIdx.x; j < 4 * L; j += blockDim.x)
        bad |= !isfinite(obs_p[j]);
    bad = __syncthreads_or(bad);
    int bad_sig = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const double sg = sig_p[s];
        bad_sig |= !(sg > 0.0 && isfinite(sg));
        w2[s] = 1.0 / (sg * sg);
    }
    return bad ? 1 : (bad_sig ? 2 : 0);
}

__global__ __launch_bounds__(kUncThreads) void k_uncert_f64(UncArgs a)
{
    __shared__ UncShared sh;
    const int L = a.ls.L;
    const int tid = threadIdx.x;
    const double inv_nu = 1.0 / (4.0 * L - GENESIS_NPAR);
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        double w2[4];
        const double *obs_p = a.obs + p * 4 * (int64_t)L;
        int st = check_pixel(obs_p, a.sigma + p * 4, L, w2);
        if (tid == 0) {
            for (int j = 0; j < GENESIS_NPAR; ++j)
                st |= !isfinite(a.p_opt[p * GENESIS_NPAR + j]);
            sh.flag = st;
        }
        __syncthreads();
        st = sh.flag;
        __syncthreads();
        const double mu = a.mu ? a.mu[p] : 1.0;
        if (tid < GENESIS_NPAR) {
            const int j = tid;
            const double q = a.p_opt[p * GENESIS_NPAR + j];
            const double span = a.hi[j] - a.lo[j];
            const double room = fmin(q - a.lo[j], a.hi[j] - q);
            double hj = a.steps[p * GENESIS_NPAR + j];
            if (!(hj >= 1e-4 * span))
                hj = 1e-4 * span;
            if (hj > 0.1 * span)
                hj = 0.1 * span;
            if (hj > 0.5 * room)
                hj = 0.5 * room;
            const int act = ((a.free_mask >> j) & 1u) && room >= 1e-4 * span;
            sh.act[j] = act;
            sh.h[j] = act ? hj : 0.0;
            sh.p[j] = q;
            if (a.steps_used)
                a.steps_used[p * GENESIS_NPAR + j] = sh.h[j];
        }
        __syncthreads();
        if (st != 0) {
            if (tid < GENESIS_NPAR) {
                a.sigma_out[p * GENESIS_NPAR + tid] = NAN;
                for (int i = 0; i < GENESIS_NPAR; ++i) {
                    if (a.hess)
                        a.hess[(p * GENESIS_NPAR + i) * GENESIS_NPAR + tid] = NAN;
                    if (a.hess_err)
                        a.hess_err[(p * GENESIS_NPAR + i) * GENESIS_NPAR + tid] = NAN;
                }
            }
            __syncthreads();
            continue;
        }
        // chi2 at the optimum: one slot with its own profiles
        if (tid == 0) {
            double x[GENESIS_NPAR];
            for (int j = 0; j < GENESIS_NPAR; ++j)
                x[j] = sh.p[j];
            model_setup(x, mu, sh.mod[0]);
            model_setup(x, mu, sh.base);
            sh.nslots = 1;
            sh.own[0] = 1;
            sh.need_base = 0;
        }
        __syncthreads();
        eval_batch<true>(a, sh, obs_p, w2, inv_nu);
        if (tid == 0)
            sh.chi2 = sh.f[0];
        // Hessian columns
        for (int j = 0; j < GENESIS_NPAR; ++j) {
            __syncthreads();
            if (!sh.act[j]) {
                if (tid < GENESIS_NPAR) {
                    sh.H[tid][j] = 0.0;
                    sh.He[tid][j] = 0.0;
                }
                continue;
            }
            tab_init(sh.out, sh.act, sh.h);
            __syncthreads();
            double t = sh.h[j];
            for (int k = 0; k < kTab && sh.out.nlive > 0; ++k, t /= kStepRatio) {
                for (int side = 0; side < 2; ++side) {
                    if (tid == 0) {
                        for (int i = 0; i < GENESIS_NPAR; ++i)
                            sh.q[i] = sh.p[i];
                        if (side == 0)
                            sh.q[j] += t;
                        else
                            sh.q[j] -= t;
                    }
                    __syncthreads();
                    gradient(a, sh, sh.out.live, side == 0 ? sh.gp : sh.gm, mu, obs_p, w2,
                             inv_nu);
                }
                if (tid < GENESIS_NPAR && sh.out.live[tid])
                    tab_row(sh.out, tid, k, (sh.gp[tid] - sh.gm[tid]) / (2.0 * t));
                __syncthreads();
                tab_count(sh.out);
                __syncthreads();
            }
            if (tid < GENESIS_NPAR) {
                sh.H[tid][j] = sh.act[tid] ? sh.out.best[tid] : 0.0;
                sh.He[tid][j] = sh.act[tid] ? sh.out.err[tid] : 0.0;
            }
        }
        __syncthreads();
        if (tid == 0) {
            for (int i = 0; i < GENESIS_NPAR; ++i)
                for (int j = i + 1; j < GENESIS_NPAR; ++j) {
                    const double s = 0.5 * (sh.H[i][j] + sh.H[j][i]);
                    sh.H[i][j] = sh.H[j][i] = s;
                    const double e = 0.5 * (sh.He[i][j] + sh.He[j][i]);
                    sh.He[i][j] = sh.He[j][i] = e;
                }
            sigmas(sh, sh.chi2, a.M, a.sigma_out + p * GENESIS_NPAR);
        }
        __syncthreads();
        if (tid < GENESIS_NPAR) {
            for (int i = 0; i < GENESIS_NPAR; ++i) {
                if (a.hess)
                    a.hess[(p * GENESIS_NPAR + i) * GENESIS_NPAR + tid] = sh.H[i][tid];
                if (a.hess_err)
                    a.hess_err[(p * GENESIS_NPAR + i) * GENESIS_NPAR + tid] = sh.He[i][tid];
            }
        }
        __syncthreads();
    }
}

// Initial steps from the final population: the RMS deviation from p_opt of
// the best max(2, pop/4) individuals (fitness order, NaN last, ties to the
// lower index), summed in rank order.  One workgroup per pixel, lane i owns
// individual i.
template <typename Real>
__global__ __launch_bounds__(1024) void k_population_steps(const uint16_t *__restrict__ genes,
                                                           const Real *__restrict__ fitness,
                                                           int64_t npix, int pop, Bounds b,
                                                           const double *__restrict__ p_opt,
                                                           double *__restrict__ steps)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Real *fit_s = reinterpret_cast<Real *>(smem);
    double *dev = reinterpret_cast<double *>(smem + ((sizeof(Real) * pop + 15) & ~(size_t)15));
    const int tid = threadIdx.x;
    const int nb = pop < 2 ? pop : (pop / 4 > 2 ? pop / 4 : 2);
    for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) {
        if (tid < pop)
            fit_s[tid] = fitness[p * pop + tid];
        __syncthreads();
        if (tid < pop) {
            const int r = fitness_rank(fit_s, pop, tid);
            if (r < nb) {
                uint32_t g[GENESIS_NPAR];
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    g[j] = genes[(p * pop + tid) * GENESIS_NPAR + j];
                double par[GENESIS_NPAR];
                decode(g, b, par);
                for (int j = 0; j < GENESIS_NPAR; ++j) {
                    const double d = par[j] - p_opt[p * GENESIS_NPAR + j];
                    dev[r * GENESIS_NPAR + j] = d * d;
                }
            }
        }
        __syncthreads();
        if (tid < GENESIS_NPAR) {
            double acc = 0.0;
            for (int r = 0; r < nb; ++r)
                acc += dev[r * GENESIS_NPAR + tid];
            steps[p * GENESIS_NPAR + tid] = sqrt(acc / nb);
        }
        __syncthreads();
    }
}

template <typename Real>
int population_steps_impl(const uint16_t *genes, const Real *fitness, int64_t npix, int32_t pop,
                          const me_bounds *bounds, const double *p_opt, double *steps,
                          void *stream)
{
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    if (pop < 1 || pop > GENESIS_MAX_POP)
        return fail(ME_EINVAL, "pop must lie in [1, %d]", GENESIS_MAX_POP);
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!genes || !fitness || !p_opt || !steps)
        return fail(ME_EINVAL, "NULL array argument");
    const int nb = pop < 2 ? pop : std::max(pop / 4, 2);
    const size_t lds = ((sizeof(Real) * pop + 15) & ~(size_t)15) + sizeof(double) * nb * GENESIS_NPAR;
    hipLaunchKernelGGL(k_population_steps<Real>, dim3(grid_for(npix)),
                       dim3(std::max(block_for_pop(pop), 64)), lds, as_stream(stream), genes,
                       fitness, npix, pop, b, p_opt, steps);
    return check_launch("ga_population_steps");
}

}  // namespace

extern "C" {

int me_uncertainty_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const double *params_opt, const double *steps,
                       uint32_t free_mask, double *sigma_params, double *hessian,
                       double *hessian_err, double *steps_used, void *stream)
{
    UncArgs a{};
    if (int rc = pack_lines(lines, grids, nlines, a.ls))
        return rc;
    if (!bounds)
        return fail(ME_EINVAL, "bounds must not be NULL");
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        if (!(bounds->hi[j] > bounds->lo[j]))
            return fail(ME_EINVAL, "uncertainties need hi > lo for every parameter (%d)", j);
        a.lo[j] = bounds->lo[j];
        a.hi[j] = bounds->hi[j];
    }
    free_mask &= 0x1ffu;
    int M = 0;
    for (int j = 0; j < GENESIS_NPAR; ++j)
        M += (free_mask >> j) & 1u;
    if (M == 0)
        return fail(ME_EINVAL, "free_mask has no free parameter");
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (4 * a.ls.L <= GENESIS_NPAR)
        return fail(ME_EINVAL, "need 4 L > 9 wavelength samples for nu > 0");
    if (npix == 0)
        return ME_OK;
    if (!obs || !sigma || !params_opt || !steps || !sigma_params)
        return fail(ME_EINVAL, "NULL array argument");
    a.obs = obs;
    a.sigma = sigma;
    a.mu = mu;
    a.p_opt = params_opt;
    a.steps = steps;
    a.npix = npix;
    a.free_mask = free_mask;
    a.M = M;
    a.sigma_out = sigma_params;
    a.hess = hessian;
    a.hess_err = hessian_err;
    a.steps_used = steps_used;
    hipLaunchKernelGGL(k_uncert_f64, dim3(grid_for(npix)), dim3(kUncThreads), 0,
                       as_stream(stream), a);
    return check_launch("me_uncertainty_f64");
}

int ga_population_steps(const uint16_t *genes, const float *fitness, int64_t npix, int32_t pop,
                        const me_bounds *bounds, const double *params_opt, double *steps,
                        void *stream)
{
    return population_steps_impl(genes, fitness, npix, pop, bounds, params_opt, steps, stream);
}

int ga_population_steps_f64(const uint16_t *genes, const double *fitness, int64_t npix,
                            int32_t pop, const me_bounds *bounds, const double *params_opt,
                            double *steps, void *stream)
{
    return population_steps_impl(genes, fitness, npix, pop, bounds, params_opt, steps, stream);
}

}  // extern "C"
