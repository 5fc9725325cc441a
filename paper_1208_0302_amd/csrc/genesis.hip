// libgenesis_hip.so: kernels and C ABI (declared in include/genesis.h).
//
// Harker & Mighell, "A GPU-Computing Approach to Solar Stokes Profile
// Inversion": genetic algorithm (Sec. 3, Algorithm 1), 16-bit genes
// (Sec. 4.2), Milne-Eddington synthesis and chi-square (Sec. 5).
//
// The paper runs only the fitness evaluation on the GPU (one block per
// individual, one thread per wavelength) and the genetic operators on the
// host.  Here the whole loop is device resident: ga_invert is one launch,
// one workgroup per pixel, one individual per lane, population and fitness
// in LDS, random numbers from a counter-based stream.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "genesis_common.h"

namespace genesis {

namespace {
thread_local std::string g_err;
}  // namespace


int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(ME_EHIP, "%s: %s", what, hipGetErrorString(e));
    return ME_OK;
}

int pack_fill(const me_fill *fill, int nlines, FillConst &fc)
{
    if (!fill)
        return fail(ME_EINVAL, "fill must not be NULL");
    if (!(fill->alpha_lo >= 0.0 && fill->alpha_lo <= fill->alpha_hi && fill->alpha_hi <= 1.0))
        return fail(ME_EINVAL, "fill fraction range [%g, %g] must lie in [0, 1]", fill->alpha_lo,
                    fill->alpha_hi);
    fc.alpha_lo = fill->alpha_lo;
    fc.alpha_hi = fill->alpha_hi;
    for (int l = 0; l < GENESIS_MAX_LINES; ++l)
        for (int k = 0; k < 4; ++k) {
            if (l < nlines && !(std::isfinite(fill->depth[l][k]) &&
                                std::isfinite(fill->width[l][k]) && std::isfinite(fill->damp[l][k])))
                return fail(ME_EINVAL, "fill coefficients of line %d must be finite", l);
            fc.depth[l][k] = fill->depth[l][k];
            fc.width[l][k] = fill->width[l][k];
            fc.damp[l][k] = fill->damp[l][k];
        }
    return ME_OK;
}

int pack_bounds(const me_bounds *b, Bounds &out)
{
    if (!b)
        return fail(ME_EINVAL, "bounds must not be NULL");
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        if (!std::isfinite(b->lo[j]) || !std::isfinite(b->hi[j]) || b->lo[j] > b->hi[j])
            return fail(ME_EINVAL, "bounds of parameter %d: need finite lo <= hi", j);
        out.lo[j] = b->lo[j];
        out.span[j] = b->hi[j] - b->lo[j];
    }
    if (!(b->lo[4] > 0))
        return fail(ME_EINVAL, "Doppler width bound must be positive");
    if (b->lo[5] < 0)
        return fail(ME_EINVAL, "damping bound must be >= 0");
    return ME_OK;
}

int pack_ga(const ga_config *cfg, GaConst &ga)
{
    if (!cfg)
        return fail(ME_EINVAL, "config must not be NULL");
    if (cfg->pop < 2 || cfg->pop > GENESIS_MAX_POP)
        return fail(ME_EINVAL, "pop = %d outside [2, %d]", cfg->pop, GENESIS_MAX_POP);
    if (cfg->tournament_k < 1 || cfg->tournament_k > std::min(cfg->pop, GENESIS_MAX_K))
        return fail(ME_EINVAL, "tournament_k = %d outside [1, min(pop, %d)]", cfg->tournament_k,
                    GENESIS_MAX_K);
    if (cfg->generations < 0)
        return fail(ME_EINVAL, "generations must be >= 0");
    const double pc = cfg->p_cross, pm = cfg->p_mut;
    if (!(pc >= 0.0 && pc <= 1.0) || !(pm >= 0.0 && pm <= 1.0))
        return fail(ME_EINVAL, "p_cross and p_mut must lie in [0, 1]");
    ga.pop = cfg->pop;
    ga.k = cfg->tournament_k;
    ga.thr_cross = (uint64_t)std::floor(pc * 4294967296.0);
    for (int kb = 0; kb < 16; ++kb) {
        double t = std::floor(2.0 * pm * (double)(kb + 1) / 17.0 * 65536.0 + 0.5);
        if (t > 65536.0)
            t = 65536.0;
        ga.mut_thr[kb] = (uint32_t)t;
    }
    ga.key.k0 = (uint32_t)(cfg->seed & 0xFFFFFFFFu);
    ga.key.k1 = (uint32_t)(cfg->seed >> 32);
    ga.pixel_base = cfg->pixel_base;
    if (cfg->n_seeded < 0 || cfg->n_seeded > cfg->pop)
        return fail(ME_EINVAL, "n_seeded = %d outside [0, pop]", cfg->n_seeded);
    if (cfg->seed_jitter < 0 || cfg->seed_jitter > 32767)
        return fail(ME_EINVAL, "seed_jitter = %d outside [0, 32767]", cfg->seed_jitter);
    if (cfg->n_seeded > 0 && !cfg->seed_params)
        return fail(ME_EINVAL, "n_seeded > 0 needs seed_params");
    if (cfg->seed_sets < 0 || cfg->seed_sets > GENESIS_MAX_POP)
        return fail(ME_EINVAL, "seed_sets = %d outside [0, %d]", cfg->seed_sets,
                    GENESIS_MAX_POP);
    if (cfg->synth_precision != GENESIS_SYNTH_NATIVE && cfg->synth_precision != GENESIS_SYNTH_FP16)
        return fail(ME_EINVAL, "synth_precision = %d is not a GENESIS_SYNTH_* value",
                    cfg->synth_precision);
    if (cfg->init_mode != 0 && cfg->init_mode != 1)
        return fail(ME_EINVAL, "init_mode = %d must be 0 (Philox) or 1 (Sobol)", cfg->init_mode);
    if (cfg->restart_every < 0)
        return fail(ME_EINVAL, "restart_every must be >= 0");
    ga.init_mode = cfg->init_mode;
    ga.restart_every = cfg->restart_every;
    ga.n_seeded = cfg->n_seeded;
    ga.seed_jitter = cfg->seed_jitter;
    ga.seed_params = cfg->n_seeded > 0 ? cfg->seed_params : nullptr;
    ga.seed_sets = cfg->seed_sets > 0 ? cfg->seed_sets : 1;
    ga.pixel_bounds = cfg->pixel_bounds;
    return ME_OK;
}


}  // namespace genesis

using namespace genesis;

namespace {

// ---- line data ---------------------------------------------------------

bool twice_int(double x, int *out)
{
    const double t = 2.0 * x, r = std::floor(t + 0.5);
    if (!std::isfinite(x) || std::fabs(t - r) > 1e-9)
        return false;
    *out = (int)r;
    return true;
}

// Relative strength of the component M_l -> M_u = M_l - q of a dipole
// transition between the lower level J_l and the upper level J_u
// (closed forms of Condon & Shortley for J_u = J_l + 1, J_l, J_l - 1;
// normalised per q group by the caller).  Arguments are doubled integers.
double cs_strength(int TJl, int TJu, int TM, int q)
{
    const double J = 0.5 * TJl, M = 0.5 * TM;
    if (TJu == TJl + 2) {
        if (q == 0)
            return (J + 1) * (J + 1) - M * M;
        if (q == -1)
            return (J + M + 1) * (J + M + 2);
        return (J - M + 1) * (J - M + 2);
    }
    if (TJu == TJl) {
        if (q == 0)
            return M * M;
        if (q == -1)
            return (J - M) * (J + M + 1);
        return (J + M) * (J - M + 1);
    }
    // J_u = J_l - 1
    if (q == 0)
        return J * J - M * M;
    if (q == -1)
        return (J - M) * (J - M - 1);
    return (J + M) * (J + M - 1);
}

// ---- kernels -----------------------------------------------------------

template <typename Real>
struct StokesSink {
    Real *out;  // [4][L] of one profile
    int L;
    __device__ __forceinline__ void operator()(int j, Real I, Real Q, Real U, Real V)
    {
        out[j] = I;
        out[L + j] = Q;
        out[2 * L + j] = U;
        out[3 * L + j] = V;
    }
};

// Stokes vectors of n models: one thread per model and chunk of
// kSynthChunk consecutive samples of one line, so that a batch of a thousand
// models still fills the chip (the model set-up is repeated per chunk).
constexpr int kSynthChunk = 8;

template <typename Real>
__host__ __device__ inline int synth_chunks(const DevLines<Real> &ls)
{
    int n = 0;
    for (int l = 0; l < ls.nlines; ++l)
        n += (ls.l[l].nlam + kSynthChunk - 1) / kSynthChunk;
    return n;
}

template <typename Real>
__global__ __launch_bounds__(256) void k_me_synth(const Real *__restrict__ params, int64_t n,
                                                  DevLines<Real> ls, int nch,
                                                  const Real *__restrict__ mu,
                                                  Real *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nch)
        return;
    const int64_t i = t / nch;
    int c = (int)(t - i * nch);
    double p[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        p[j] = (double)params[i * GENESIS_NPAR + j];
    Model<Real> m;
    model_setup(p, mu ? (double)mu[i] : 1.0, m);
    StokesSink<Real> s{out + i * 4 * (int64_t)ls.L, ls.L};
#pragma unroll
    for (int l = 0; l < GENESIS_MAX_LINES; ++l) {
        if (l >= ls.nlines)
            return;
        const DevLine<Real> &ln = ls.l[l];
        const int cl = (ln.nlam + kSynthChunk - 1) / kSynthChunk;
        if (c < cl) {
            const int j0 = c * kSynthChunk;
            synth_line_range(m, ln, s, j0, min(j0 + kSynthChunk, ln.nlam));
            return;
        }
        c -= cl;
    }
}

// Stokes vectors with the FP16 profile synthesis of ga_invert's
// GENESIS_SYNTH_FP16 mode (one thread per model).
__global__ __launch_bounds__(256) void k_me_synth_h(const float *__restrict__ params, int64_t n,
                                                    DevLines<float> ls, DevLinesH lh,
                                                    const float *__restrict__ mu,
                                                    float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double p[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        p[j] = (double)params[i * GENESIS_NPAR + j];
    ModelH m;
    model_setup(p, mu ? (double)mu[i] : 1.0, m);
    StokesSink<float> s{out + i * 4 * (int64_t)ls.L, ls.L};
    synthesize_h(m, ls, lh, s);
}

// Fitness of every individual of every pixel: from params (me_chi2) or from
// genes through the decoding operator (ga_evaluate).
template <typename Real, bool FROM_GENES>
__global__ __launch_bounds__(1024) void k_fitness(const Real *__restrict__ params,
                                                  const uint16_t *__restrict__ genes, Bounds b,
                                                  int64_t npix, int pop,
                                                  const Real *__restrict__ obs,
                                                  const Real *__restrict__ sigma,
                                                  const Real *__restrict__ mu, DevLines<Real> ls,
                                                  Real *__restrict__ out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Vec4<Real> *obs_s = reinterpret_cast<Vec4<Real> *>(smem);
    const int L = ls.L;
    const Real inv_nu = (Real)(1.0 / (4.0 * L - GENESIS_NPAR));
    for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) {
        Real w2[4];
        const int st = stage_pixel(obs + p * 4 * (int64_t)L, sigma + p * 4, L, obs_s, w2);
        const double m_mu = mu ? (double)mu[p] : 1.0;
        for (int i = threadIdx.x; i < pop; i += blockDim.x) {
            double par[GENESIS_NPAR];
            const int64_t row = (p * pop + i) * GENESIS_NPAR;
            if (FROM_GENES) {
                uint32_t g[GENESIS_NPAR];
#pragma unroll
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    g[j] = genes[row + j];
                decode(g, b, par);
            } else {
#pragma unroll
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    par[j] = (double)params[row + j];
            }
            Real c = (Real)NAN;
            if (st == 0) {
                Model<Real> m;
                model_setup(par, m_mu, m);
                c = chi2_of(m, ls, obs_s, w2, inv_nu);
            }
            out[p * pop + i] = c;
        }
        __syncthreads();
    }
}

__global__ void k_ga_init(int64_t npix, GaConst ga, Bounds b, uint16_t *__restrict__ genes)
{
    const int pop = ga.pop;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npix * pop)
        return;
    const int64_t p = t / pop;
    const int i = (int)(t - p * pop);
    uint32_t g[GENESIS_NPAR];
    Bounds box;
    stage_box(b, ga.pixel_bounds, p, box);
    initial_genes(ga.pixel_base + (uint32_t)p, p, i, ga, box, g);
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        genes[t * GENESIS_NPAR + j] = (uint16_t)g[j];
}

// Restart of generation t (workgroup per pixel): ranks by fitness, the worst
// half replaced by Sobol points, the rest copied.
template <typename Real>
__global__ __launch_bounds__(1024) void k_ga_restart(const uint16_t *__restrict__ genes_in,
                                                     const Real *__restrict__ fitness,
                                                     int64_t npix, GaConst ga, int t,
                                                     uint16_t *__restrict__ genes_out)
{
    extern __shared__ __align__(16) unsigned char smem[];
    Real *fit_s = reinterpret_cast<Real *>(smem);
    const int pop = ga.pop;
    const int tid = threadIdx.x;
    for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) {
        for (int i = tid; i < pop; i += blockDim.x)
            fit_s[i] = fitness[p * pop + i];
        __syncthreads();
        const uint32_t pix = ga.pixel_base + (uint32_t)p;
        for (int i = tid; i < pop; i += blockDim.x) {
            const int64_t row = (p * pop + i) * GENESIS_NPAR;
            uint32_t g[GENESIS_NPAR];
            if (!restart_genes(ga, pix, t, fitness_rank(fit_s, pop, i), g))
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    g[j] = genes_in[row + j];
            for (int j = 0; j < GENESIS_NPAR; ++j)
                genes_out[row + j] = (uint16_t)g[j];
        }
        __syncthreads();
    }
}

template <typename Real>
__global__ void k_decode(const uint16_t *__restrict__ genes, int64_t n, Bounds b,
                         Real *__restrict__ params)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t g[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        g[j] = genes[i * GENESIS_NPAR + j];
    double p[GENESIS_NPAR];
    decode(g, b, p);
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        params[i * GENESIS_NPAR + j] = (Real)p[j];
}

// Child sink writing the step outputs to global memory.
struct GlobalChild {
    uint16_t *genes, *masks;  // row of this child [9]
    int32_t *parents, *xpoint;
    __device__ __forceinline__ void meta(int a, int b, int x)
    {
        if (parents) {
            parents[0] = a;
            parents[1] = b;
        }
        if (xpoint)
            *xpoint = x;
    }
    __device__ __forceinline__ void gene(int j, uint32_t g, uint32_t m)
    {
        genes[j] = (uint16_t)g;
        if (masks)
            masks[j] = (uint16_t)m;
    }
};

template <typename Real>
struct StepArgs {
    const uint16_t *genes_in;
    const Real *fitness;
    int64_t npix;
    uint32_t gen;
    GaConst ga;
    uint16_t *genes_out;
    int32_t *parents, *xpoint, *elite;
    uint16_t *masks;
};

template <typename Real>
__global__ __launch_bounds__(1024) void k_ga_step(StepArgs<Real> a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int pop = a.ga.pop;
    const GaLds<Real> s = ga_lds<Real>(smem, 0, pop);
    const int tid = threadIdx.x;
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        for (int i = tid; i < pop; i += blockDim.x) {
            s.fit[i] = a.fitness[p * pop + i];
#pragma unroll
            for (int j = 0; j < GENESIS_NPAR; ++j)
                s.genes[j * pop + i] = a.genes_in[(p * pop + i) * GENESIS_NPAR + j];
        }
        __syncthreads();
        const int e = block_argmin(s.fit, pop, s.red_f, s.red_i);
        const uint32_t pix = a.ga.pixel_base + (uint32_t)p;
        if (tid < pop) {
            const int64_t row = p * pop + tid;
            GlobalChild out{a.genes_out + row * GENESIS_NPAR,
                            a.masks ? a.masks + row * GENESIS_NPAR : nullptr,
                            a.parents ? a.parents + row * 2 : nullptr,
                            a.xpoint ? a.xpoint + row : nullptr};
            if (tid == 0) {
                out.meta(e, e, 0);
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    out.gene(j, s.genes[j * pop + e], 0u);
                if (a.elite)
                    a.elite[p] = e;
            } else {
                make_child(tid, pix, a.gen, s.fit, s.genes, a.ga, out);
            }
        }
        __syncthreads();
    }
}

template <int SYN>
struct SynLines {};
template <>
struct SynLines<GENESIS_SYNTH_FP16> {
    DevLinesH lh;
};

// fill-fraction constants and output, present in the fill kernels only
template <typename Real, bool FILL>
struct FillArgs {
};
template <typename Real>
struct FillArgs<Real, true> {
    FillConst fc;
    Real *best_alpha;
};

template <typename Real, int SYN = GENESIS_SYNTH_NATIVE, bool FILL = false>
struct InvertArgs : SynLines<SYN>, FillArgs<Real, FILL> {
    const Real *obs, *sigma, *mu;
    int64_t npix;
    int32_t generations;
    DevLines<Real> ls;
    Bounds b;
    GaConst ga;
    Real *best_params, *best_chi2, *final_fitness;
    int32_t *status;
    uint16_t *final_genes;
    // > 0 when every workgroup of the launch is resident at once: the number
    // of CUs
    int32_t prio_mate;
};

// Progress counters of single-round launches, one per XCD (workgroup b runs
// on XCD b mod 8), 256 bytes apart; zeroed by k_progress_reset before each
// such launch.  Launches that overlap on one device share them, which can
// only change the issue order, never a result.
constexpr int kProgressStride = 32;
__device__ unsigned long long g_ga_progress[8 * kProgressStride];

__global__ void k_progress_reset()
{
    if (threadIdx.x < 8)
        g_ga_progress[threadIdx.x * kProgressStride] = 0ull;
}

// The whole of Algorithm 1 for one pixel per workgroup: the population
// lives in LDS (two buffers: parents and children), lane i owns
// individual i.
template <typename Real, int SYN, bool FILL>
__global__ __launch_bounds__(1024) void k_ga_invert(InvertArgs<Real, SYN, FILL> a)
{
    code_shift<FILL ? (sizeof(Real) == 8 ? GENESIS_PAD_FILL_F64
                                         : SYN == GENESIS_SYNTH_FP16 ? GENESIS_PAD_FILL_F16
                                                                     : GENESIS_PAD_FILL_F32)
                    : SYN == GENESIS_SYNTH_FP16
                          ? GENESIS_PAD_INVERT_F16
                          : (sizeof(Real) == 8 ? GENESIS_PAD_INVERT_F64 : GENESIS_PAD_INVERT_F32)>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int pop = a.ga.pop;
    const int L = a.ls.L;
    const GaLds<Real> s = ga_lds<Real>(smem, L, pop);
    const int tid = threadIdx.x;
    const bool active = tid < pop;
    // nu = 4L - 9, or 4L - 10 with the fill fraction as a tenth parameter
    const Real inv_nu = (Real)(1.0 / (4.0 * L - (FILL ? GENESIS_NPAR + 1 : GENESIS_NPAR)));
    FillPix<Real> &fp = *reinterpret_cast<FillPix<Real> *>(s.fill);
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        const double mu = a.mu ? (double)a.mu[p] : 1.0;
        if (tid == 0) {
            stage_box(a.b, a.ga.pixel_bounds, p, *s.box);
            if constexpr (FILL)
                fill_setup(a.fc, a.ls.nlines, mu, fp);
        }
        Real w2[4];
        int st = stage_pixel(a.obs + p * 4 * (int64_t)L, a.sigma + p * 4, L, s.obs, w2);
        if (st == 0 && a.ga.pixel_bounds)
            st = box_status(*s.box, SYN == GENESIS_SYNTH_FP16);
        if constexpr (FILL)
            if (st == 0)
                st = fp.status;
        if (st != 0) {
            if (tid == 0) {
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    a.best_params[p * GENESIS_NPAR + j] = (Real)NAN;
                a.best_chi2[p] = (Real)NAN;
                if (a.status)
                    a.status[p] = st;
                if constexpr (FILL)
                    a.best_alpha[p] = (Real)NAN;
            }
            if (active) {
                if (a.final_fitness)
                    a.final_fitness[p * pop + tid] = (Real)NAN;
                if (a.final_genes)
                    for (int j = 0; j < GENESIS_NPAR; ++j)
                        a.final_genes[(p * pop + tid) * GENESIS_NPAR + j] = 0;
            }
            __syncthreads();
            continue;
        }
        const uint32_t pix = a.ga.pixel_base + (uint32_t)p;
        GenState<Real> gs = generation_zero(s, pop, tid, pix, p, a.ga);
        // In a launch that is resident all at once, a SIMD issues oldest
        // first, so the first-dispatched workgroups run ahead and finish
        // early and the launch ends on SIMDs holding one or two waves.
        // Raising the priority of the workgroups that lag their XCD's average
        // generation keeps their progress even.  It changes the issue order
        // only, never a result.
        unsigned long long *progress =
            a.prio_mate > 0 ? g_ga_progress + kProgressStride * (blockIdx.x & 7) : nullptr;
        generation_loop(s, pop, tid, pix, a.ga, a.generations, a.generations, progress, gs,
                        [&](const uint16_t *genes) -> Real {
                            if constexpr (FILL && SYN == GENESIS_SYNTH_FP16) {
                                float al;
                                return evaluate_fill_h(genes, pop, tid, *s.box, mu, a.ls, a.lh,
                                                       fp, (float)a.fc.alpha_lo,
                                                       (float)a.fc.alpha_hi, s.obs, w2, inv_nu,
                                                       al);
                            } else if constexpr (FILL) {
                                Real al;
                                return evaluate_fill(genes, pop, tid, *s.box, mu, a.ls, fp,
                                                     (Real)a.fc.alpha_lo, (Real)a.fc.alpha_hi,
                                                     s.obs, w2, inv_nu, al);
                            } else if constexpr (SYN == GENESIS_SYNTH_FP16) {
                                return evaluate_lds_h(genes, pop, tid, *s.box, mu, a.ls, a.lh,
                                                      s.obs, w2, inv_nu);
                            } else {
                                return evaluate_lds(genes, pop, tid, *s.box, mu, a.ls, s.obs, w2,
                                                    inv_nu);
                            }
                        });
        double par[GENESIS_NPAR];
        const int e = best_of(s, pop, gs, par);
        if (tid == 0) {
            for (int j = 0; j < GENESIS_NPAR; ++j)
                a.best_params[p * GENESIS_NPAR + j] = (Real)par[j];
            a.best_chi2[p] = s.fit[e];
            if constexpr (FILL && SYN == GENESIS_SYNTH_FP16) {
                // the best individual's alpha: the same evaluation again
                ModelH m;
                model_setup(par, mu, m);
                float al;
                (void)chi2_fill_of_h(m, a.ls, a.lh, fp, (float)a.fc.alpha_lo,
                                     (float)a.fc.alpha_hi, s.obs, w2, inv_nu, al);
                a.best_alpha[p] = al;
            } else if constexpr (FILL) {
                Model<Real> m;
                model_setup(par, mu, m);
                Real al;
                (void)chi2_fill_of(m, a.ls, fp, (Real)a.fc.alpha_lo, (Real)a.fc.alpha_hi, s.obs,
                                   w2, inv_nu, al);
                a.best_alpha[p] = al;
            }
            if (a.status)
                a.status[p] = 0;
        }
        const int cur = gs.cur;
        const Real f = gs.f;
        if (active) {
            if (a.final_fitness)
                a.final_fitness[p * pop + tid] = f;
            if (a.final_genes)
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    a.final_genes[(p * pop + tid) * GENESIS_NPAR + j] = s.genes[cur + j * pop + tid];
        }
        __syncthreads();
    }
}


// ---- inverse-max weights (Sec. 5.4) -------------------------------------
//
// sigma = 1 / w per pixel and Stokes parameter: for I the span of the
// observed I over every sample of the pixel (continuum minus line core), for
// Q, U, V the largest magnitude; each at least `floor`; NaN for all four when
// a sample of the pixel is not finite.  One wavefront per pixel; max and min
// are exact, so the result does not depend on the reduction order.
template <typename Real>
__global__ __launch_bounds__(64) void k_invmax_sigma(const Real *__restrict__ obs, int64_t npix,
                                                     int L, Real floor, Real *__restrict__ sigma)
{
    for (int64_t p = blockIdx.x; p < npix; p += gridDim.x) {
        const Real *o = obs + p * 4 * (int64_t)L;
        Real imax = -INFINITY, imin = INFINITY, q = 0, u = 0, v = 0;
        int bad = 0;
        for (int j = threadIdx.x; j < L; j += 64) {
            const Real I = o[j], Q = o[L + j], U = o[2 * L + j], V = o[3 * L + j];
            bad |= !(isfinite(I) && isfinite(Q) && isfinite(U) && isfinite(V));
            imax = fmax(imax, I);
            imin = fmin(imin, I);
            q = fmax(q, fabs(Q));
            u = fmax(u, fabs(U));
            v = fmax(v, fabs(V));
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            imax = fmax(imax, __shfl_xor(imax, off));
            imin = fmin(imin, __shfl_xor(imin, off));
            q = fmax(q, __shfl_xor(q, off));
            u = fmax(u, __shfl_xor(u, off));
            v = fmax(v, __shfl_xor(v, off));
            bad |= __shfl_xor(bad, off);
        }
        if (threadIdx.x == 0) {
            Real *s = sigma + p * 4;
            if (bad) {
                s[0] = s[1] = s[2] = s[3] = (Real)NAN;
            } else {
                s[0] = fmax(imax - imin, floor);
                s[1] = fmax(q, floor);
                s[2] = fmax(u, floor);
                s[3] = fmax(v, floor);
            }
        }
    }
}

// ---- heuristic first guesses (Sec. 5.5 seeds) ---------------------------
//
// One workgroup of 256 per pixel, FP64.  Per line (x the offset of a sample
// from the rest wavelength, I_c the largest I of the pixel, d = I_c - I,
// d+- = I_c - (I +- V), I'' the central second difference, 0 at the ends,
// C = 4.6686e-13 lambda0^2, gbar the first moment of the red sigma group):
// v = c (sum x d / sum d) / lambda0; B_par from the centres of gravity of d+
// and d-, (x+ - x-) / (2 C gbar); weak-field (q, u) = -4 (sum Q I'', sum U I'')
// / (C^2 gbar^2 sum I''^2); half-depth width hw = step #{d >= max d / 2} / 2;
// core depth 1 - min I / I_c.  Lines are combined with weights W = step sum d
// (times gbar for B_par, gbar^2 for q, u); B_perp = sqrt(hypot(q, u)),
// azimuth = atan2(u, q) / 2, B = hypot(B_par, B_perp), inclination =
// atan2(B_perp, B_par); mu S1 = 3/4 I_c, S0 = I_c / 4, eta0 = D'/(1 - D') for
// D' = min(D / 0.75, 0.97), Doppler width hw / sqrt(ln(eta0 + 2)), damping
// the middle of its range; a non-finite estimate becomes the middle of its
// range; all clamped into the box.
constexpr int kGuessThreads = 256;
constexpr int kGuessSums = 10;  // per line: s0 s1 sp0 sp1 sm0 sm1 sQ sU s2 cnt

struct GuessArgs {
    const double *obs, *mu;
    int64_t npix;
    DevLines<double> ls;
    double gbar[GENESIS_MAX_LINES];
    double lo[GENESIS_NPAR], hi[GENESIS_NPAR];
    float *params;
};

__device__ double guess_reduce(double v, bool take_max, double *red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = take_max ? fmax(v, o) : v + o;
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[w] = v;
    __syncthreads();
    double t = red[0];
    for (int k = 1; k < kGuessThreads / 64; ++k)
        t = take_max ? fmax(t, red[k]) : t + red[k];
    return t;
}

// Stokes vector of models with a fill fraction (Sec. 5.2), one thread per
// model and sample: alpha M + (1 - alpha) I_c N e.  A model whose field-free
// profile is invalid at its mu gets NaN.
template <typename Real>
__global__ void k_me_synth_fill(const Real *__restrict__ params, const Real *__restrict__ alpha,
                                int64_t n, DevLines<Real> ls, const Real *__restrict__ mu,
                                FillConst fc, Real *__restrict__ out)
{
    const int L = ls.L;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * L)
        return;
    const int64_t i = t / L;
    const int j = (int)(t - i * L);
    int l = 0;
    while (l + 1 < ls.nlines && j >= ls.l[l + 1].off)
        ++l;
    const DevLine<Real> &ln = ls.l[l];
    const int jj = j - ln.off;
    double par[GENESIS_NPAR];
    for (int k = 0; k < GENESIS_NPAR; ++k)
        par[k] = (double)params[i * GENESIS_NPAR + k];
    const double mu_i = mu ? (double)mu[i] : 1.0;
    Real *o = out + i * 4 * (int64_t)L;
    FillLine<Real> f;
    if (!fill_setup_line(fc, l, mu_i, f)) {
        o[j] = o[L + j] = o[2 * L + j] = o[3 * L + j] = (Real)NAN;
        return;
    }
    Model<Real> m;
    model_setup(par, mu_i, m);
    Real I, Q, U, V;
    stokes_at(m, ln, jj, I, Q, U, V);
    const Real x = fma(ln.step, (Real)jj, ln.off0);
    const Real N = fma(-f.scale, fill_h(f, (x - m.vlos * ln.dop_kms) * f.inv_w), (Real)1);
    const Real a = alpha[i];
    o[j] = fma(a, I, ((Real)1 - a) * ((m.S0 + m.muS1) * N));
    o[L + j] = a * Q;
    o[2 * L + j] = a * U;
    o[3 * L + j] = a * V;
}

template <typename Real>
int synth_fill_impl(const Real *params, const Real *alpha, int64_t n, const me_line *lines,
                    const me_grid *grids, int32_t nlines, const Real *mu, const me_fill *fill,
                    Real *stokes, void *stream)
{
    DevLines<Real> ls;
    if (int rc = pack_lines(lines, grids, nlines, ls))
        return rc;
    FillConst fc;
    if (int rc = pack_fill(fill, nlines, fc))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!params || !alpha || !stokes)
        return fail(ME_EINVAL, "params, alpha and stokes must not be NULL");
    const int bs = 256;
    const int64_t blocks = (n * ls.L + bs - 1) / bs;
    if (blocks > kMaxGrid)
        return fail(ME_EINVAL, "n too large");
    hipLaunchKernelGGL(k_me_synth_fill<Real>, dim3((unsigned)blocks), dim3(bs), 0,
                       as_stream(stream), params, alpha, n, ls, mu, fc, stokes);
    return check_launch("me_synth_fill");
}

// ---- per-pixel search boxes (Sec. 5.3 pre-fit ranges, Sec. 5.5 polarity)

struct BoxArgs {
    const double *obs, *sigma, *prefit;
    int64_t npix;
    DevLines<double> ls;
    double lo[GENESIS_NPAR], hi[GENESIS_NPAR];
    double nsigma;
    float *box;
};

__device__ __forceinline__ double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// One workgroup per pixel: the first moment of V about each line's centre of
// gravity (of I_c - I) decides the polarity; thread 0 applies the pre-fit
// ranges and writes the box.
__global__ __launch_bounds__(kGuessThreads) void k_search_box(BoxArgs a)
{
    __shared__ double red[kGuessThreads / 64];
    const int L = a.ls.L;
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        const double *I = a.obs + p * 4 * (int64_t)L, *V = I + 3 * L;
        double lo[GENESIS_NPAR], hi[GENESIS_NPAR];
#pragma unroll
        for (int j = 0; j < GENESIS_NPAR; ++j) {
            lo[j] = a.lo[j];
            hi[j] = a.hi[j];
        }
        if (a.nsigma > 0.0) {
            double m = -INFINITY;
            for (int j = threadIdx.x; j < L; j += kGuessThreads)
                m = fmax(m, I[j]);
            const double Ic = guess_reduce(m, true, red);
            double sV = 0.0, sxx = 0.0;
            for (int l = 0; l < a.ls.nlines; ++l) {
                const DevLine<double> &ln = a.ls.l[l];
                double d0 = 0.0, d1 = 0.0;
                for (int j = threadIdx.x; j < ln.nlam; j += kGuessThreads) {
                    const double d = Ic - I[ln.off + j];
                    d0 += d;
                    d1 += (ln.off0 + ln.step * j) * d;
                }
                const double xc = guess_reduce(d1, false, red) / guess_reduce(d0, false, red);
                double m1 = 0.0, m2 = 0.0;
                for (int j = threadIdx.x; j < ln.nlam; j += kGuessThreads) {
                    const double x = ln.off0 + ln.step * j - xc;
                    m1 += x * V[ln.off + j];
                    m2 += x * x;
                }
                sV += guess_reduce(m1, false, red);
                sxx += guess_reduce(m2, false, red);
            }
            const double noise = a.sigma[p * 4 + 3] * sqrt(sxx);
            // V's first moment is negative for inclinations below 90 degrees
            if (fabs(sV) > a.nsigma * noise) {
                if (sV > 0.0 && a.hi[1] >= 90.0)
                    lo[1] = fmax(a.lo[1], 90.0);
                else if (sV < 0.0 && a.lo[1] <= 90.0)
                    hi[1] = fmin(a.hi[1], 90.0);
            }
        }
        if (threadIdx.x == 0) {
            if (a.prefit) {
                const double *f = a.prefit + p * GENESIS_NPAR;
                // a non-magnetic fit absorbs Zeeman broadening into the
                // Doppler width and the damping: upper bounds
                if (isfinite(f[4]))
                    hi[4] = clampd(1.1 * f[4], a.lo[4], a.hi[4]);
                if (isfinite(f[5]))
                    hi[5] = clampd(1.5 * f[5] + 0.1 * (a.hi[5] - a.lo[5]), a.lo[5], a.hi[5]);
                // eta0 and S1 (beta0): multiplicative windows
                if (isfinite(f[6]) && f[6] > 0.0) {
                    lo[6] = clampd(f[6] / 8.0, a.lo[6], a.hi[6]);
                    hi[6] = clampd(f[6] * 8.0, a.lo[6], a.hi[6]);
                }
                if (isfinite(f[8]) && f[8] > 0.0) {
                    lo[8] = clampd(f[8] / 1.5, a.lo[8], a.hi[8]);
                    hi[8] = clampd(f[8] * 1.5, a.lo[8], a.hi[8]);
                }
            }
            float *out = a.box + p * 2 * GENESIS_NPAR;
            for (int j = 0; j < GENESIS_NPAR; ++j) {
                out[j] = (float)lo[j];
                out[GENESIS_NPAR + j] = (float)hi[j];
            }
        }
        __syncthreads();
    }
}

// The first guesses of one pixel (all threads call; the result is valid on
// thread 0): g9 clamped into the common box, and the centre-of-gravity
// longitudinal field before any clamping.
__device__ void first_guess_pixel(const GuessArgs &a, int64_t p, double *red,
                                  double (&g9)[GENESIS_NPAR], double &bpar_cog)
{
    const int L = a.ls.L;
    const double *I = a.obs + p * 4 * (int64_t)L, *Q = I + L, *U = I + 2 * L, *V = I + 3 * L;
    double m = -INFINITY;
    for (int j = threadIdx.x; j < L; j += kGuessThreads)
        m = fmax(m, I[j]);
    const double Ic = guess_reduce(m, true, red);
    double W = 0, Wv = 0, Wg = 0, WgB = 0, Wg2 = 0, Wq = 0, Wu = 0, Whw = 0, depth = 0;
    for (int l = 0; l < a.ls.nlines; ++l) {
        const DevLine<double> &ln = a.ls.l[l];
        const double *Il = I + ln.off;
        double mx = -INFINITY;
        for (int j = threadIdx.x; j < ln.nlam; j += kGuessThreads)
            mx = fmax(mx, Ic - Il[j]);
        const double dmax = guess_reduce(mx, true, red);
        double acc[kGuessSums] = {};
        for (int j = threadIdx.x; j < ln.nlam; j += kGuessThreads) {
            const double x = ln.off0 + ln.step * j;
            const double i0 = Il[j], v = V[ln.off + j];
            const double d = Ic - i0, dp = Ic - (i0 + v), dm = Ic - (i0 - v);
            const double d2 = (j > 0 && j + 1 < ln.nlam)
                                  ? (Il[j + 1] - 2.0 * i0 + Il[j - 1]) / (ln.step * ln.step)
                                  : 0.0;
            acc[0] += d;
            acc[1] += x * d;
            acc[2] += dp;
            acc[3] += x * dp;
            acc[4] += dm;
            acc[5] += x * dm;
            acc[6] += Q[ln.off + j] * d2;
            acc[7] += U[ln.off + j] * d2;
            acc[8] += d2 * d2;
            acc[9] += d >= 0.5 * dmax ? 1.0 : 0.0;
        }
        double tot[kGuessSums];
#pragma unroll
        for (int k = 0; k < kGuessSums; ++k)
            tot[k] = guess_reduce(acc[k], false, red);
        const double lam0 = ln.dop_kms * kCkms;
        const double C = kZeeman * lam0 * lam0, g = a.gbar[l];
        const double xc = tot[1] / tot[0];
        const double bpar = (tot[3] / tot[2] - tot[5] / tot[4]) / (2.0 * C * g);
        const double qq = -4.0 * tot[6] / (C * C * g * g * tot[8]);
        const double uu = -4.0 * tot[7] / (C * C * g * g * tot[8]);
        const double hw = 0.5 * ln.step * tot[9];
        const double Wl = ln.step * tot[0];
        W += Wl;
        Wv += Wl * kCkms * xc / lam0;
        Wg += Wl * g;
        WgB += Wl * g * bpar;
        Wg2 += Wl * g * g;
        Wq += Wl * g * g * qq;
        Wu += Wl * g * g * uu;
        Whw += Wl * hw;
        depth = fmax(depth, dmax / Ic);
    }
    const double bpar = WgB / Wg, q = Wq / Wg2, u = Wu / Wg2;
    bpar_cog = bpar;
    const double bperp = sqrt(hypot(q, u));
    double azim = 0.5 * atan2(u, q) * (180.0 / kPi);
    azim = fmod(azim + 180.0, 180.0);
    const double Dp = fmin(depth / 0.75, 0.97);
    const double eta0 = Dp / (1.0 - Dp);
    const double mu = a.mu ? a.mu[p] : 1.0;
    const double raw[GENESIS_NPAR] = {hypot(bpar, bperp),
                                      atan2(bperp, bpar) * (180.0 / kPi),
                                      azim,
                                      Wv / W,
                                      Whw / W / sqrt(log(eta0 + 2.0)),
                                      0.5 * (a.lo[5] + a.hi[5]),
                                      eta0,
                                      0.25 * Ic,
                                      0.75 * Ic / mu};
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        const double v = isfinite(raw[j]) ? raw[j] : 0.5 * (a.lo[j] + a.hi[j]);
        g9[j] = fmin(fmax(v, a.lo[j]), a.hi[j]);
    }
}

__global__ __launch_bounds__(kGuessThreads) void k_first_guess(GuessArgs a)
{
    __shared__ double red[kGuessThreads / 64];
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        double g9[GENESIS_NPAR], bpar;
        first_guess_pixel(a, p, red, g9, bpar);
        if (threadIdx.x == 0)
            for (int j = 0; j < GENESIS_NPAR; ++j)
                a.params[p * GENESIS_NPAR + j] = (float)g9[j];
        __syncthreads();
    }
}

// ---- the four separate seeds of Sec. 5.5 ---------------------------------
//
// Per pixel, with the thermodynamic estimates of the first guesses (v_los,
// Doppler width, damping, eta0, S0, S1) shared by all four, per line I', I''
// the differences of the first guesses (I' one-sided at the window ends),
// cg = C gbar and a = cg^2, summed over every line's samples:
//  0 weak field: B_par = -sum cg V I' / sum (cg I')^2, q = -4 sum a Q I'' /
//    sum (a I'')^2 (u likewise), B_perp = sqrt(hypot(q, u)), azimuth
//    atan2(u, q) / 2;
//  1 integral relations: |B_par| = sum |V| / sum cg |I'| with the sign of
//    -sum cg V I', B_perp = sqrt(4 sum sqrt(Q^2 + U^2) / sum a |I''|), and
//    the azimuth chi0 = atan2(2 sum Q U, sum (Q^2 - U^2)) / 4 or chi0 + 90
//    deg, the one whose projection Q cos 2chi + U sin 2chi over the three
//    samples around each line's minimum of I is not positive;
//  2 centre of gravity: B = |B_par| of the first guesses, inclination 0 (B_par
//    >= 0) or 180, azimuth unseeded (NaN);
//  3 non-magnetic: B = 0, both angles unseeded;
// B = hypot(B_par, B_perp), inclination atan2(B_perp, B_par) for 0 and 1.
// Then, in the pixel's box (pixel_bounds, else the common box): a non-finite
// B or thermodynamic value becomes the middle of the box, the azimuth is
// wrapped into [0, 180), an inclination outside the box becomes 180 minus
// itself, and every seeded value is clamped into the box.
constexpr int kSeedSums = 13;

struct SeedArgs {
    GuessArgs g;
    const float *box;  // [npix][2][9] or nullptr
    float *seeds;      // [npix][4][9]
};

__global__ __launch_bounds__(kGuessThreads) void k_seeds(SeedArgs sa)
{
    const GuessArgs &a = sa.g;
    __shared__ double red[kGuessThreads / 64];
    const int L = a.ls.L;
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        double g9[GENESIS_NPAR], bcog;
        first_guess_pixel(a, p, red, g9, bcog);
        const double *I = a.obs + p * 4 * (int64_t)L, *Q = I + L, *U = I + 2 * L, *V = I + 3 * L;
        double tot[kSeedSums] = {};
        for (int l = 0; l < a.ls.nlines; ++l) {
            const DevLine<double> &ln = a.ls.l[l];
            const int n = ln.nlam;
            const double *Il = I + ln.off;
            // the line's minimum of I, first sample on ties
            double mn = -INFINITY;
            for (int j = threadIdx.x; j < n; j += kGuessThreads)
                mn = fmax(mn, -Il[j]);
            mn = guess_reduce(mn, true, red);
            double ci = -INFINITY;
            for (int j = threadIdx.x; j < n; j += kGuessThreads)
                if (-Il[j] == mn)
                    ci = fmax(ci, -(double)j);
            const int c = (int)(-guess_reduce(ci, true, red));
            const double lam0 = ln.dop_kms * kCkms;
            const double C = kZeeman * lam0 * lam0, cg = C * a.gbar[l], aa = cg * cg;
            const double st = ln.step;
            double acc[kSeedSums] = {};
            for (int j = threadIdx.x; j < n; j += kGuessThreads) {
                const double i0 = Il[j], q = Q[ln.off + j], u = U[ln.off + j], v = V[ln.off + j];
                const double d1 = j == 0       ? (Il[1] - Il[0]) / st
                                  : j == n - 1 ? (Il[n - 1] - Il[n - 2]) / st
                                               : (Il[j + 1] - Il[j - 1]) / (2.0 * st);
                const double d2 = (j > 0 && j + 1 < n) ? (Il[j + 1] - 2.0 * i0 + Il[j - 1]) / (st * st)
                                                       : 0.0;
                acc[0] += v * d1;
                acc[1] += (cg * d1) * (cg * d1);
                acc[2] += q * d2;
                acc[3] += u * d2;
                acc[4] += (aa * d2) * (aa * d2);
                acc[5] += fabs(v);
                acc[6] += fabs(d1);
                acc[7] += sqrt(q * q + u * u);
                acc[8] += fabs(d2);
                acc[9] += q * u;
                acc[10] += q * q - u * u;
                if (j >= c - 1 && j <= c + 1) {
                    acc[11] += q;
                    acc[12] += u;
                }
            }
            double t[kSeedSums];
#pragma unroll
            for (int k = 0; k < kSeedSums; ++k)
                t[k] = guess_reduce(acc[k], false, red);
            tot[0] += t[0] * cg;
            tot[1] += t[1];
            tot[2] += aa * t[2];
            tot[3] += aa * t[3];
            tot[4] += t[4];
            tot[5] += t[5];
            tot[6] += cg * t[6];
            tot[7] += t[7];
            tot[8] += aa * t[8];
            tot[9] += t[9];
            tot[10] += t[10];
            tot[11] += t[11];
            tot[12] += t[12];
        }
        if (threadIdx.x == 0) {
            const double r2d = 180.0 / kPi;
            double blo[GENESIS_NPAR], bhi[GENESIS_NPAR];
            for (int j = 0; j < GENESIS_NPAR; ++j) {
                blo[j] = sa.box ? (double)sa.box[(p * 2) * GENESIS_NPAR + j] : a.lo[j];
                bhi[j] = sa.box ? (double)sa.box[(p * 2 + 1) * GENESIS_NPAR + j] : a.hi[j];
            }
            // weak field
            const double bpar = -tot[0] / tot[1];
            const double q = -4.0 * tot[2] / tot[4], u = -4.0 * tot[3] / tot[4];
            const double bperp = sqrt(hypot(q, u));
            // integral relations
            const double ipar = fabs(tot[5] / tot[6]) * (-tot[0] >= 0.0 ? 1.0 : -1.0);
            const double iperp = sqrt(4.0 * tot[7] / tot[8]);
            double chi0 = 0.25 * atan2(2.0 * tot[9], tot[10]);
            if (tot[11] * cos(2.0 * chi0) + tot[12] * sin(2.0 * chi0) > 0.0)
                chi0 += 0.5 * kPi;
            const double mag[4][3] = {
                {hypot(bpar, bperp), atan2(bperp, bpar) * r2d, 0.5 * atan2(u, q) * r2d},
                {hypot(ipar, iperp), atan2(iperp, ipar) * r2d, chi0 * r2d},
                {fabs(bcog), bcog >= 0.0 ? 0.0 : 180.0, NAN},
                {0.0, NAN, NAN}};
            for (int k = 0; k < 4; ++k) {
                double v[GENESIS_NPAR];
                for (int j = 0; j < 3; ++j)
                    v[j] = mag[k][j];
                for (int j = 3; j < GENESIS_NPAR; ++j)
                    v[j] = g9[j];
                bool seeded[GENESIS_NPAR];
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    seeded[j] = !isnan(v[j]);
                seeded[0] = true;
                if (!isfinite(v[0]))
                    v[0] = 0.5 * (blo[0] + bhi[0]);
                for (int j = 1; j <= 2; ++j)
                    if (seeded[j] && !isfinite(v[j]))
                        v[j] = 0.5 * (blo[j] + bhi[j]);
                if (seeded[2]) {
                    v[2] = fmod(v[2], 180.0);
                    if (v[2] < 0.0)
                        v[2] += 180.0;
                }
                if (seeded[1] && !(blo[1] <= v[1] && v[1] <= bhi[1]))
                    v[1] = 180.0 - v[1];
                for (int j = 3; j < GENESIS_NPAR; ++j)
                    if (!isfinite(v[j]))
                        v[j] = 0.5 * (blo[j] + bhi[j]);
                float *o = sa.seeds + (p * 4 + k) * GENESIS_NPAR;
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    o[j] = seeded[j] ? (float)fmin(fmax(v[j], blo[j]), bhi[j]) : NAN;
            }
        }
        __syncthreads();
    }
}

// ---- FP64 Levenberg-Marquardt refinement --------------------------------
//
// One workgroup of kRefineThreads per pixel; thread t takes samples t,
// t + kRefineThreads, ... of every line, so with the 128-sample lines of the
// slit workload every thread holds one sample of each line (the 12- and the
// 3-component one) and no wavefront idles at the reductions.  In
// normalised coordinates x_j = (p_j - lo_j)/(hi_j - lo_j) in [0, 1]: forward
// differences with step h = 1e-7 (backwards at the upper edge) give the
// Jacobian; A = J^T J and g = J^T r are reduced over the workgroup; thread 0
// solves (A + lambda diag(A)) d = g by Cholesky (d_j = 0 where A_jj = 0);
// the trial x' = clamp(x + d) is accepted if chi2 drops (lambda /= 10, floor
// 1e-12), else lambda *= 10 (cap 1e12), at most 10 trials per iteration;
// lambda starts at 1e-3; the loop stops after an iteration without an
// accepted trial.
//
// With the fill fraction (Sec. 5.2) the model is alpha M + (1 - alpha) I_c N e
// and alpha in [alpha_lo, alpha_hi] is a tenth coordinate fitted the same
// way (nu = 4L - 10).
//
// The normal equations are a Gram matrix, [J r]^T [J r], so they go to the
// FP64 matrix cores: each thread forms its sample's four weighted Jacobian
// rows (one per Stokes parameter) and residuals in registers; one Stokes
// parameter at a time, every wavefront writes its 64 rows to LDS and
// accumulates them with 16 v_mfma_f64_16x16x4 (4 rows each; lane l supplies
// row l / 16, column l % 16 as both operands, the columns past the residual
// read as 0).  The 16 x 16 accumulator of each wavefront holds J^T J, J^T r
// (and r^T r) of its rows; the wavefronts' accumulators are added in
// wavefront order.
constexpr int kRefineThreads = 128;
constexpr int kRefineWaves = kRefineThreads / 64;

typedef double v4f64 __attribute__((ext_vector_type(4)));

template <bool FILL>
struct RefineDims {
    static constexpr int NP = GENESIS_NPAR + (FILL ? 1 : 0);  // fitted coordinates
    static constexpr int NC = NP + 1;                         // + the residual column
};

struct RefineArgs {
    const double *obs, *sigma, *mu, *params_in;
    int64_t npix;
    int32_t iterations;
    DevLines<double> ls;
    double lo[GENESIS_NPAR], span[GENESIS_NPAR];
    double *params_out, *chi2_out;
    int32_t *iters_done;
    uint32_t free_mask;  // bit j: coordinate j is adjusted (held otherwise)
    int32_t zero_field;  // start (and, with bit 0 clear, hold) B at 0
    // fill fraction
    FillConst fc;
    const double *alpha_in;
    double *alpha_out;
};

template <bool FILL>
struct RefineShared {
    static constexpr int NP = RefineDims<FILL>::NP, NC = RefineDims<FILL>::NC;
    Model<double> jm[GENESIS_NPAR + 1];  // models at x and at x + h_k e_k (Jacobian)
    double x[NP], xt[NP];
    double alpha[NP + 1];                // fill: alpha of each of those models
    double red[kRefineWaves];
    double rows[kRefineWaves][64 * NC];  // one Stokes parameter's rows per wavefront
    double gram[kRefineWaves][NP][NC];   // each wavefront's J^T [J r]
    double nrm[NP][NC];                  // J^T J and J^T r at x
    double lam, chi2;
    FillPix<double> fp;
    int flag;
};

__device__ __forceinline__ void model_from_x(const RefineArgs &a, const double *x, double mu,
                                             Model<double> &m)
{
    double p[GENESIS_NPAR];
#pragma unroll
    for (int j = 0; j < GENESIS_NPAR; ++j)
        p[j] = a.lo[j] + a.span[j] * x[j];
    model_setup(p, mu, m);
}

__device__ __forceinline__ double alpha_of(const RefineArgs &a, double x)
{
    return a.fc.alpha_lo + (a.fc.alpha_hi - a.fc.alpha_lo) * x;
}

// Sum of one per-thread value over the workgroup (fixed order: wavefront
// butterflies, then wavefronts in index order); every thread gets it.
template <bool FILL>
__device__ __forceinline__ double block_sum1(double v, RefineShared<FILL> &sh)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0)
        sh.red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kRefineWaves; ++k)
        t += sh.red[k];
    __syncthreads();
    return t;
}

// Field-free profile N of line ln at sample jj for line-of-sight velocity vlos.
__device__ __forceinline__ double fill_n(const FillLine<double> &f, const DevLine<double> &ln,
                                         int jj, double vlos)
{
    const double xw = fma(ln.step, (double)jj, ln.off0);
    return fma(-f.scale, fill_h(f, (xw - vlos * ln.dop_kms) * f.inv_w), 1.0);
}

// alpha M + (1 - alpha) I_c N e in place.
__device__ __forceinline__ void fill_mix(double al, double ic, double N, double (&M)[4])
{
    M[0] = fma(al, M[0], (1.0 - al) * (ic * N));
    M[1] *= al;
    M[2] *= al;
    M[3] *= al;
}

// chi2 * nu contribution of this thread's wavelengths at normalised x
template <bool FILL>
__device__ __forceinline__ double chi2_part(const RefineArgs &a, const RefineShared<FILL> &sh,
                                            const double *x, double mu,
                                            const Vec4<double> *obs_s, const double (&w2)[4])
{
    Model<double> m;
    model_from_x(a, x, mu, m);
    const double al = FILL ? alpha_of(a, x[GENESIS_NPAR]) : 1.0;
    double acc = 0.0;
    for (int l = 0; l < a.ls.nlines; ++l) {
        const DevLine<double> &ln = a.ls.l[l];
        for (int jj = threadIdx.x; jj < ln.nlam; jj += kRefineThreads) {
            double M[4];
            stokes_at(m, ln, jj, M[0], M[1], M[2], M[3]);
            if constexpr (FILL)
                fill_mix(al, m.S0 + m.muS1, fill_n(sh.fp.l[l], ln, jj, m.vlos), M);
            const Vec4<double> o = obs_s[ln.off + jj];
            const double dI = o.x - M[0], dQ = o.y - M[1], dU = o.z - M[2], dV = o.w - M[3];
            acc += w2[0] * dI * dI + w2[1] * dQ * dQ + w2[2] * dU * dU + w2[3] * dV * dV;
        }
    }
    return acc;
}

template <int N>
__device__ bool cholesky_n(double (&M)[N][N], const double (&g)[N], double (&d)[N])
{
    double Lm[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = M[i][j];
            for (int k = 0; k < j; ++k)
                s -= Lm[i][k] * Lm[j][k];
            if (i == j) {
                if (!(s > 0.0))
                    return false;
                Lm[i][i] = sqrt(s);
            } else {
                Lm[i][j] = s / Lm[j][j];
            }
        }
    double y[N];
    for (int i = 0; i < N; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k)
            s -= Lm[i][k] * y[k];
        y[i] = s / Lm[i][i];
    }
    for (int i = N - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < N; ++k)
            s -= Lm[k][i] * d[k];
        d[i] = s / Lm[i][i];
    }
    return true;
}

// Group profiles (h, l of blue, pi, red) at sample jj of the base model jm[0]
// (pr[0], accumulated as profiles_at does) and of the four models that move
// the Faddeeva arguments z = v + i a: jm[1] (B), jm[4] (v_los), jm[5]
// (Doppler width), jm[6] (damping) (pr[1..4]), each component's w taken to
// first order about its base value,
//   w(z) ~ w(z0) + w'(z0) (z - z0),  w'(z) = -2 z w(z) + 2 i / sqrt(pi),
// so one Faddeeva evaluation per component serves all five models.
__device__ __forceinline__ void profiles_lin(const Model<double> *jm, const DevLine<double> &ln,
                                             int jj, double (&pr)[5][6])
{
    const int mi[5] = {0, 1, 4, 5, 6};
    double x0[5], zb[5], da[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const Model<double> &m = jm[mi[q]];
        const double xb = (ln.off0 - m.vlos * ln.dop_kms) * m.inv_dop;
        x0[q] = fma((double)jj, ln.step * m.inv_dop, xb);
        zb[q] = ln.zee_G * m.B * m.inv_dop;
        da[q] = m.a - jm[0].a;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            pr[q][i] = 0.0;
    }
    const double a0 = jm[0].a;
    const int lim[4] = {0, ln.nb, ln.nb + ln.np, ln.nb + ln.np + ln.nr};
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        for (int c = lim[g]; c < lim[g + 1]; ++c) {
            const double s = ln.s[c], w = ln.w[c];
            const double v0 = fma(-s, zb[0], x0[0]);
            double H, L;
            voigt_f64(a0, v0, H, L);
            const double dr = -2.0 * fma(v0, H, -(a0 * L));
            const double di = fma(-2.0, fma(v0, L, a0 * H), 1.1283791670955125739);  // 2/sqrt(pi)
            pr[0][2 * g] = fma(w, H, pr[0][2 * g]);
            pr[0][2 * g + 1] = fma(w, L, pr[0][2 * g + 1]);
#pragma unroll
            for (int q = 1; q < 5; ++q) {
                const double dv = fma(-s, zb[q], x0[q]) - v0;
                pr[q][2 * g] = fma(w, H + fma(dr, dv, -(di * da[q])), pr[q][2 * g]);
                pr[q][2 * g + 1] = fma(w, L + fma(di, dv, dr * da[q]), pr[q][2 * g + 1]);
            }
        }
    }
}

// The weighted Jacobian rows J[k][s] (k < NP) and residuals r[s] of one sample
// (zero when the thread has no sample).
template <bool FILL>
__device__ __forceinline__ void jacobian_rows(const RefineArgs &a, const RefineShared<FILL> &sh,
                                              int l, int jj, const double (&hx)[RefineDims<FILL>::NP],
                                              const double (&sig)[4], const Vec4<double> *obs_s,
                                              double (&J)[RefineDims<FILL>::NP][4], double (&r)[4])
{
    constexpr int NP = RefineDims<FILL>::NP;
    const DevLine<double> &ln = a.ls.l[l];
    double M0[4], pl[5][6], N0 = 1.0;
    profiles_lin(sh.jm, ln, jj, pl);
    const double(&pr0)[6] = pl[0];
    unno_rachkovsky(sh.jm[0], pr0[0], pr0[1], pr0[2], pr0[3], pr0[4], pr0[5], M0[0], M0[1],
                    M0[2], M0[3]);
    double Mm[4] = {M0[0], M0[1], M0[2], M0[3]};  // magnetic part of the base model
    if constexpr (FILL) {
        N0 = fill_n(sh.fp.l[l], ln, jj, sh.jm[0].vlos);
        fill_mix(sh.alpha[0], sh.jm[0].S0 + sh.jm[0].muS1, N0, M0);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        double Mk[4];
        if (!((a.free_mask >> k) & 1u)) {
            // a held coordinate: zero column, so A_kk = 0 and d_k = 0
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                J[k][s4] = 0.0;
            continue;
        }
        if (k == GENESIS_NPAR) {
            // alpha (fill only): the base model mixed at the perturbed alpha
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                Mk[s4] = Mm[s4];
            fill_mix(sh.alpha[k + 1], sh.jm[0].S0 + sh.jm[0].muS1, N0, Mk);
        } else {
            const Model<double> &mk = sh.jm[k + 1];
            if (k == 0 || (k >= 3 && k <= 5)) {
                // B, v_los, Doppler width, damping: the linearised profiles
                const double(&pq)[6] = pl[k == 0 ? 1 : k - 1];
                unno_rachkovsky(mk, pq[0], pq[1], pq[2], pq[3], pq[4], pq[5], Mk[0], Mk[1],
                                Mk[2], Mk[3]);
            } else {
                // the angles, eta0, S0, S1 leave every Voigt argument
                // unchanged: the base profiles, the perturbed algebra
                unno_rachkovsky(mk, pr0[0], pr0[1], pr0[2], pr0[3], pr0[4], pr0[5], Mk[0],
                                Mk[1], Mk[2], Mk[3]);
            }
            if constexpr (FILL)
                fill_mix(sh.alpha[0], mk.S0 + mk.muS1,
                         k == 3 ? fill_n(sh.fp.l[l], ln, jj, mk.vlos) : N0, Mk);
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            J[k][s4] = (Mk[s4] - M0[s4]) / (hx[k] * sig[s4]);
    }
    const Vec4<double> o = obs_s[ln.off + jj];
    r[0] = (o.x - M0[0]) / sig[0];
    r[1] = (o.y - M0[1]) / sig[1];
    r[2] = (o.z - M0[2]) / sig[2];
    r[3] = (o.w - M0[3]) / sig[3];
}

template <bool FILL>
__global__ __launch_bounds__(kRefineThreads) void k_refine_f64(RefineArgs a)
{
    constexpr int NP = RefineDims<FILL>::NP, NC = RefineDims<FILL>::NC;
    static_assert(NC <= 16, "the Gram matrix fits one 16 x 16 accumulator");
    code_shift<GENESIS_PAD_REFINE>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = a.ls.L;
    Vec4<double> *obs_s = reinterpret_cast<Vec4<double> *>(smem);
    __shared__ RefineShared<FILL> sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double inv_nu = 1.0 / (4.0 * L - NP);
    const double h = 1e-7;
    for (int64_t p = blockIdx.x; p < a.npix; p += gridDim.x) {
        const double mu = a.mu ? a.mu[p] : 1.0;
        if constexpr (FILL)
            if (tid == 0)
                fill_setup(a.fc, a.ls.nlines, mu, sh.fp);
        double w2[4];
        int st = stage_pixel(a.obs + p * 4 * (int64_t)L, a.sigma + p * 4, L, obs_s, w2);
        if constexpr (FILL)
            if (st == 0)
                st = sh.fp.status;
        if (st != 0) {
            if (tid == 0) {
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    a.params_out[p * GENESIS_NPAR + j] = NAN;
                if constexpr (FILL)
                    a.alpha_out[p] = NAN;
                a.chi2_out[p] = NAN;
                if (a.iters_done)
                    a.iters_done[p] = 0;
            }
            __syncthreads();
            continue;
        }
        const double sig[4] = {a.sigma[p * 4], a.sigma[p * 4 + 1], a.sigma[p * 4 + 2],
                               a.sigma[p * 4 + 3]};
        if (tid < GENESIS_NPAR) {
            const double pin = (a.zero_field && tid == 0) ? 0.0 : a.params_in[p * GENESIS_NPAR + tid];
            const double v = (pin - a.lo[tid]) / a.span[tid];
            sh.x[tid] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
        }
        if constexpr (FILL)
            if (tid == GENESIS_NPAR) {
                const double v =
                    (a.alpha_in[p] - a.fc.alpha_lo) / (a.fc.alpha_hi - a.fc.alpha_lo);
                sh.x[GENESIS_NPAR] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
        if (tid == 0)
            sh.lam = 1e-3;
        __syncthreads();
        {
            const double c = block_sum1(chi2_part(a, sh, sh.x, mu, obs_s, w2), sh);
            if (tid == 0)
                sh.chi2 = c;
            __syncthreads();
        }
        int it = 0;
        for (; it < a.iterations; ++it) {
            // ---- Jacobian and normal equations
            double hx[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j)
                hx[j] = (sh.x[j] + h <= 1.0) ? h : -h;
            // the model at x (slot 0) and the nine forward-difference models
            // (slot k + 1), set up once per iteration for every wavelength
            if (tid <= GENESIS_NPAR) {
                double xk[GENESIS_NPAR];
#pragma unroll
                for (int j = 0; j < GENESIS_NPAR; ++j)
                    xk[j] = sh.x[j] + (j == tid - 1 ? hx[j] : 0.0);
                model_from_x(a, xk, mu, sh.jm[tid]);
            }
            if constexpr (FILL)
                if (tid == 0)
                    for (int k = 0; k <= NP; ++k)
                        sh.alpha[k] = alpha_of(a, sh.x[GENESIS_NPAR] +
                                                      (k == NP ? hx[GENESIS_NPAR] : 0.0));
            __syncthreads();
            v4f64 acc = {0.0, 0.0, 0.0, 0.0};
            const int rrow = lane >> 4, rcol = lane & 15;
            for (int l = 0; l < a.ls.nlines; ++l) {
                const int nlam = a.ls.l[l].nlam;
                for (int c0 = 0; c0 < nlam; c0 += kRefineThreads) {
                    const int jj = c0 + tid;
                    double J[NP][4], r[4];
                    if (jj < nlam) {
                        jacobian_rows<FILL>(a, sh, l, jj, hx, sig, obs_s, J, r);
                    } else {
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) {
                            r[s4] = 0.0;
#pragma unroll
                            for (int k = 0; k < NP; ++k)
                                J[k][s4] = 0.0;
                        }
                    }
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        double *rw = sh.rows[wv];
#pragma unroll
                        for (int k = 0; k < NP; ++k)
                            rw[lane * NC + k] = J[k][s4];
                        rw[lane * NC + NP] = r[s4];
                        __syncthreads();
#pragma unroll 4
                        for (int t = 0; t < 16; ++t) {
                            const double v = rcol < NC ? rw[(4 * t + rrow) * NC + rcol] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
                        }
                        __syncthreads();
                    }
                }
            }
            // accumulator element v of lane l: row l / 16 + 4 v, column l % 16
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = rrow + 4 * v;
                if (i < NP && rcol < NC)
                    sh.gram[wv][i][rcol] = acc[v];
            }
            __syncthreads();
            for (int e = tid; e < NP * NC; e += kRefineThreads) {
                double t = 0.0;
                for (int w = 0; w < kRefineWaves; ++w)
                    t += sh.gram[w][e / NC][e % NC];
                sh.nrm[e / NC][e % NC] = t;
            }
            __syncthreads();
            // ---- damped trials
            bool accepted = false;
            for (int trial = 0; trial < 10; ++trial) {
                if (tid == 0) {
                    double Mx[NP][NP], g[NP], d[NP];
                    for (int i = 0; i < NP; ++i)
                        for (int j = i; j < NP; ++j)
                            Mx[i][j] = Mx[j][i] = sh.nrm[i][j];
                    for (int i = 0; i < NP; ++i)
                        g[i] = sh.nrm[i][NP];
                    for (int i = 0; i < NP; ++i) {
                        const double aii = Mx[i][i];
                        if (aii == 0.0) {
                            for (int j = 0; j < NP; ++j)
                                Mx[i][j] = Mx[j][i] = 0.0;
                            Mx[i][i] = 1.0;
                            g[i] = 0.0;
                        } else {
                            Mx[i][i] = aii + sh.lam * aii;
                        }
                    }
                    sh.flag = cholesky_n<NP>(Mx, g, d) ? 1 : 0;
                    if (sh.flag)
                        for (int j = 0; j < NP; ++j) {
                            const double v = sh.x[j] + d[j];
                            sh.xt[j] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
                        }
                    else
                        sh.lam = fmin(sh.lam * 10.0, 1e12);
                }
                __syncthreads();
                if (!sh.flag) {
                    __syncthreads();
                    continue;
                }
                const double c = block_sum1(chi2_part(a, sh, sh.xt, mu, obs_s, w2), sh);
                if (tid == 0) {
                    if (c < sh.chi2) {
                        for (int j = 0; j < NP; ++j)
                            sh.x[j] = sh.xt[j];
                        sh.chi2 = c;
                        sh.lam = fmax(sh.lam / 10.0, 1e-12);
                        sh.flag = 2;
                    } else {
                        sh.lam = fmin(sh.lam * 10.0, 1e12);
                    }
                }
                __syncthreads();
                accepted = sh.flag == 2;
                __syncthreads();
                if (accepted)
                    break;
            }
            if (!accepted)
                break;
        }
        if (tid < GENESIS_NPAR)
            a.params_out[p * GENESIS_NPAR + tid] = a.lo[tid] + a.span[tid] * sh.x[tid];
        if (tid == 0) {
            if constexpr (FILL)
                a.alpha_out[p] = alpha_of(a, sh.x[GENESIS_NPAR]);
            a.chi2_out[p] = sh.chi2 * inv_nu;
            if (a.iters_done)
                a.iters_done[p] = it;
        }
        __syncthreads();
    }
}

// ---- host wrappers -----------------------------------------------------

template <typename Real>
int synth_impl(const Real *params, int64_t n, const me_line *lines, const me_grid *grids,
               int nlines, const Real *mu, Real *stokes, void *stream)
{
    DevLines<Real> ls;
    if (int rc = pack_lines(lines, grids, nlines, ls))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!params || !stokes)
        return fail(ME_EINVAL, "params and stokes must not be NULL");
    const int nch = synth_chunks(ls);
    const int bs = 256;
    const int64_t blocks = (n * nch + bs - 1) / bs;
    if (n > ((int64_t)1 << 40) / nch || blocks > kMaxGrid)
        return fail(ME_EINVAL, "n too large");
    hipLaunchKernelGGL(k_me_synth<Real>, dim3((unsigned)blocks), dim3(bs), 0, as_stream(stream),
                       params, n, ls, nch, mu, stokes);
    return check_launch("me_synth");
}

template <typename Real, bool FROM_GENES>
int fitness_impl(const Real *params, const uint16_t *genes, const me_bounds *bounds, int64_t npix,
                 int pop, const Real *obs, const Real *sigma, const Real *mu,
                 const me_line *lines, const me_grid *grids, int nlines, Real *out, void *stream)
{
    DevLines<Real> ls;
    if (int rc = pack_lines(lines, grids, nlines, ls))
        return rc;
    Bounds b{};
    if (FROM_GENES)
        if (int rc = pack_bounds(bounds, b))
            return rc;
    if (npix < 0 || pop < 1 || pop > GENESIS_MAX_POP)
        return fail(ME_EINVAL, "npix >= 0 and 1 <= pop <= %d required", GENESIS_MAX_POP);
    if (4 * ls.L <= GENESIS_NPAR)
        return fail(ME_EINVAL, "need 4 L > 9 wavelength samples for nu > 0");
    if (npix == 0)
        return ME_OK;
    if (!(FROM_GENES ? (const void *)genes : (const void *)params) || !obs || !sigma || !out)
        return fail(ME_EINVAL, "NULL array argument");
    const size_t lds = sizeof(Vec4<Real>) * (size_t)ls.L;
    if (lds > kMaxLds)
        return fail(ME_ENOMEM, "observation of %d samples exceeds LDS", ls.L);
    hipLaunchKernelGGL((k_fitness<Real, FROM_GENES>), dim3(grid_for(npix)),
                       dim3(block_for_pop(pop)), lds, as_stream(stream), params, genes, b, npix,
                       pop, obs, sigma, mu, ls, out);
    return check_launch("fitness");
}

template <typename Real>
int step_impl(const uint16_t *genes_in, const Real *fitness, int64_t npix, const ga_config *cfg,
              int32_t generation, uint16_t *genes_out, int32_t *parents, int32_t *xpoint,
              uint16_t *masks, int32_t *elite, void *stream)
{
    StepArgs<Real> a{};
    if (int rc = pack_ga(cfg, a.ga))
        return rc;
    if (generation < 1)
        return fail(ME_EINVAL, "generation must be >= 1 (generation 0 is ga_init)");
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!genes_in || !fitness || !genes_out)
        return fail(ME_EINVAL, "NULL array argument");
    const size_t bytes = (size_t)npix * cfg->pop * GENESIS_NPAR * sizeof(uint16_t);
    const char *gi = (const char *)genes_in, *go = (const char *)genes_out;
    if (gi < go + bytes && go < gi + bytes)
        return fail(ME_EINVAL, "genes_in and genes_out overlap");
    a.genes_in = genes_in;
    a.fitness = fitness;
    a.npix = npix;
    a.gen = (uint32_t)generation;
    a.genes_out = genes_out;
    a.parents = parents;
    a.xpoint = xpoint;
    a.masks = masks;
    a.elite = elite;
    const size_t lds = ga_lds_bytes<Real>(0, cfg->pop);
    hipLaunchKernelGGL(k_ga_step<Real>, dim3(grid_for(npix)), dim3(block_for_pop(cfg->pop)), lds,
                       as_stream(stream), a);
    return check_launch("ga_step");
}

// The number of CUs when all `nblocks` workgroups of `kernel` fit on the
// device at once (occupancy at this block size and LDS), else 0.  A failed
// query only turns the progress-based issue priority off.
int single_round_stride(const void *kernel, int block, size_t lds, int64_t nblocks)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return ncu > 0 && per_cu > 0 && nblocks <= (int64_t)ncu * per_cu ? ncu : 0;
}

template <typename Real, int SYN, bool FILL = false>
int invert_impl(const Real *obs, const Real *sigma, const Real *mu, int64_t npix,
                const me_line *lines, const me_grid *grids, int nlines, const me_bounds *bounds,
                const ga_config *cfg, Real *best_params, Real *best_chi2, int32_t *status,
                uint16_t *final_genes, Real *final_fitness, void *stream,
                const me_fill *fill = nullptr, Real *best_alpha = nullptr)
{
    InvertArgs<Real, SYN, FILL> a{};
    if (int rc = pack_lines(lines, grids, nlines, a.ls))
        return rc;
    if (int rc = pack_bounds(bounds, a.b))
        return rc;
    if (int rc = pack_ga(cfg, a.ga))
        return rc;
    if (SYN == GENESIS_SYNTH_FP16 && !(bounds->lo[5] >= 0.0 && bounds->hi[5] <= kHalfMaxDamping))
        return fail(ME_EINVAL, "FP16 synthesis needs damping bounds within [0, %g]",
                    kHalfMaxDamping);
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (4 * a.ls.L <= GENESIS_NPAR + (FILL ? 1 : 0))
        return fail(ME_EINVAL, "need 4 L > %d wavelength samples for nu > 0",
                    GENESIS_NPAR + (FILL ? 1 : 0));
    if constexpr (FILL) {
        if (int rc = pack_fill(fill, nlines, a.fc))
            return rc;
        if (npix > 0 && !best_alpha)
            return fail(ME_EINVAL, "best_alpha must not be NULL");
        a.best_alpha = best_alpha;
    }
    const size_t lds = ga_lds_bytes<Real>(a.ls.L, cfg->pop);
    if (lds > kMaxLds)
        return fail(ME_ENOMEM, "L = %d, pop = %d need %zu B of LDS (> %zu)", a.ls.L, cfg->pop,
                    lds, kMaxLds);
    if (npix == 0)
        return ME_OK;
    if (!obs || !sigma || !best_params || !best_chi2)
        return fail(ME_EINVAL, "NULL array argument");
    a.obs = obs;
    a.sigma = sigma;
    a.mu = mu;
    a.npix = npix;
    a.generations = cfg->generations;
    a.best_params = best_params;
    a.best_chi2 = best_chi2;
    a.status = status;
    a.final_genes = final_genes;
    a.final_fitness = final_fitness;
    if constexpr (SYN == GENESIS_SYNTH_FP16)
        pack_lines_h(a.ls, a.lh);
    a.prio_mate = single_round_stride((const void *)k_ga_invert<Real, SYN, FILL>,
                                      block_for_pop(cfg->pop), lds, npix);
    if (a.prio_mate > 0)
        hipLaunchKernelGGL(k_progress_reset, dim3(1), dim3(64), 0, as_stream(stream));
    hipLaunchKernelGGL((k_ga_invert<Real, SYN, FILL>), dim3(grid_for(npix)),
                       dim3(block_for_pop(cfg->pop)), lds, as_stream(stream), a);
    return check_launch("ga_invert");
}

template <typename Real>
int invert_dispatch(const Real *obs, const Real *sigma, const Real *mu, int64_t npix,
                    const me_line *lines, const me_grid *grids, int nlines,
                    const me_bounds *bounds, const ga_config *cfg, Real *best_params,
                    Real *best_chi2, int32_t *status, uint16_t *final_genes, Real *final_fitness,
                    void *stream)
{
    if (!cfg)
        return fail(ME_EINVAL, "config must not be NULL");
    if (cfg->synth_precision == GENESIS_SYNTH_NATIVE)
        return invert_impl<Real, GENESIS_SYNTH_NATIVE>(obs, sigma, mu, npix, lines, grids, nlines,
                                                       bounds, cfg, best_params, best_chi2,
                                                       status, final_genes, final_fitness, stream);
    if constexpr (std::is_same<Real, float>::value) {
        if (cfg->synth_precision == GENESIS_SYNTH_FP16)
            return invert_impl<float, GENESIS_SYNTH_FP16>(obs, sigma, mu, npix, lines, grids,
                                                          nlines, bounds, cfg, best_params,
                                                          best_chi2, status, final_genes,
                                                          final_fitness, stream);
    }
    return fail(ME_EINVAL, "synth_precision = %d not available for this entry point",
                cfg->synth_precision);
}


template <bool FILL>
int refine_impl(const double *obs, const double *sigma, const double *mu, int64_t npix,
                const me_line *lines, const me_grid *grids, int nlines, const me_bounds *bounds,
                const double *params_in, int iterations, double *params_out, double *chi2_out,
                int32_t *iters_done, void *stream, uint32_t free_mask = 0x1ffu,
                bool zero_field = false, const me_fill *fill = nullptr,
                const double *alpha_in = nullptr, double *alpha_out = nullptr)
{
    constexpr int NP = RefineDims<FILL>::NP;
    RefineArgs a{};
    if (int rc = pack_lines(lines, grids, nlines, a.ls))
        return rc;
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        if (!(b.span[j] > 0))
            return fail(ME_EINVAL, "refinement needs hi > lo for every parameter (%d)", j);
        a.lo[j] = b.lo[j];
        a.span[j] = b.span[j];
    }
    if constexpr (FILL) {
        if (int rc = pack_fill(fill, nlines, a.fc))
            return rc;
        if (!(a.fc.alpha_hi > a.fc.alpha_lo))
            return fail(ME_EINVAL, "refinement needs alpha_hi > alpha_lo");
    }
    if (iterations < 0)
        return fail(ME_EINVAL, "iterations must be >= 0");
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (4 * a.ls.L <= NP)
        return fail(ME_EINVAL, "need 4 L > %d wavelength samples for nu > 0", NP);
    const size_t lds = sizeof(Vec4<double>) * (size_t)a.ls.L;
    if (lds + sizeof(RefineShared<FILL>) > kMaxLds)
        return fail(ME_ENOMEM, "observation of %d samples exceeds LDS", a.ls.L);
    if (npix == 0)
        return ME_OK;
    if (!obs || !sigma || !params_in || !params_out || !chi2_out)
        return fail(ME_EINVAL, "NULL array argument");
    if (FILL && (!alpha_in || !alpha_out))
        return fail(ME_EINVAL, "NULL alpha array");
    a.obs = obs;
    a.sigma = sigma;
    a.mu = mu;
    a.params_in = params_in;
    a.npix = npix;
    a.iterations = iterations;
    a.params_out = params_out;
    a.chi2_out = chi2_out;
    a.iters_done = iters_done;
    a.free_mask = free_mask & ((1u << NP) - 1u);
    a.zero_field = zero_field ? 1 : 0;
    a.alpha_in = alpha_in;
    a.alpha_out = alpha_out;
    hipLaunchKernelGGL(k_refine_f64<FILL>, dim3(grid_for(npix)), dim3(kRefineThreads), lds,
                       as_stream(stream), a);
    return check_launch(FILL ? "me_refine_fill_f64" : "me_refine_f64");
}
}  // namespace

// ---- C ABI -------------------------------------------------------------

template <typename Real>
int restart_impl(const uint16_t *genes_in, const Real *fitness, int64_t npix,
                 const ga_config *cfg, int32_t generation, uint16_t *genes_out, void *stream)
{
    GaConst ga;
    if (int rc = pack_ga(cfg, ga))
        return rc;
    if (ga.restart_every < 1 || generation < 1 || generation % ga.restart_every != 0)
        return fail(ME_EINVAL, "generation %d is not a restart generation (restart_every %d)",
                    generation, ga.restart_every);
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!genes_in || !fitness || !genes_out)
        return fail(ME_EINVAL, "NULL array argument");
    const size_t bytes = (size_t)npix * cfg->pop * GENESIS_NPAR * sizeof(uint16_t);
    const char *gi = (const char *)genes_in, *go = (const char *)genes_out;
    if (gi < go + bytes && go < gi + bytes)
        return fail(ME_EINVAL, "genes_in and genes_out overlap");
    hipLaunchKernelGGL(k_ga_restart<Real>, dim3(grid_for(npix)), dim3(block_for_pop(cfg->pop)),
                       sizeof(Real) * cfg->pop, as_stream(stream), genes_in, fitness, npix, ga,
                       (int)generation, genes_out);
    return check_launch("ga_restart");
}


namespace {

template <typename Real>
int invmax_impl(const Real *obs, int64_t npix, const me_grid *grids, int32_t nlines, double floor,
                Real *sigma, void *stream)
{
    if (!grids || nlines < 1 || nlines > GENESIS_MAX_LINES)
        return fail(ME_EINVAL, "need 1..%d grids", GENESIS_MAX_LINES);
    int64_t L = 0;
    for (int l = 0; l < nlines; ++l) {
        if (grids[l].n < 1)
            return fail(ME_EINVAL, "grid %d has %d samples", l, grids[l].n);
        L += grids[l].n;
    }
    if (L > (1 << 28))
        return fail(ME_EINVAL, "%lld samples per pixel are too many", (long long)L);
    if (!(floor >= 0.0) || !std::isfinite(floor))
        return fail(ME_EINVAL, "floor must be finite and >= 0");
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!obs || !sigma)
        return fail(ME_EINVAL, "NULL array argument");
    hipLaunchKernelGGL(k_invmax_sigma<Real>, dim3(grid_for(npix)), dim3(64), 0, as_stream(stream),
                       obs, npix, (int)L, (Real)floor, sigma);
    return check_launch("me_invmax_sigma");
}

int pack_guess(const double *obs, const double *mu, int64_t npix, const me_line *lines,
               const me_grid *grids, int32_t nlines, const me_bounds *bounds, GuessArgs &a)
{
    if (int rc = pack_lines(lines, grids, nlines, a.ls))
        return rc;
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    for (int l = 0; l < nlines; ++l) {
        double g = 0.0;
        for (int c = 0; c < lines[l].ncomp; ++c)
            if (lines[l].q[c] == 1)
                g += (double)lines[l].strength[c] * (double)lines[l].shift[c];
        if (!(g > 0.0))
            return fail(ME_EINVAL, "line %d has no Zeeman splitting (first moment of the red "
                                   "sigma group %g)", l, g);
        a.gbar[l] = g;
        if (grids[l].n < 3)
            return fail(ME_EINVAL, "line %d: need at least 3 samples", l);
    }
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        a.lo[j] = bounds->lo[j];
        a.hi[j] = bounds->hi[j];
    }
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    a.obs = obs;
    a.mu = mu;
    a.npix = npix;
    return ME_OK;
}

}  // namespace

extern "C" {

const char *me_last_error(void) { return g_err.c_str(); }

int genesis_abi_version(void) { return GENESIS_ABI_VERSION; }

size_t genesis_struct_size(int32_t which)
{
    switch (which) {
    case 0: return sizeof(me_line);
    case 1: return sizeof(me_grid);
    case 2: return sizeof(me_bounds);
    case 3: return sizeof(ga_config);
    case 4: return sizeof(me_fill);
    default: return 0;
    }
}

int me_line_from_terms(double lambda0_A, double Jl, double gl, double Ju, double gu,
                       me_line *out)
{
    if (!out)
        return fail(ME_EINVAL, "out must not be NULL");
    int TJl, TJu;
    if (!twice_int(Jl, &TJl) || !twice_int(Ju, &TJu) || TJl < 0 || TJu < 0)
        return fail(ME_EINVAL, "J values must be non-negative integers or half-integers");
    if (std::abs(TJl - TJu) > 2 || ((TJl - TJu) & 1) || (TJl == 0 && TJu == 0))
        return fail(ME_EINVAL, "J_l = %g -> J_u = %g is not a dipole transition", Jl, Ju);
    if (!(lambda0_A > 0) || !std::isfinite(gl) || !std::isfinite(gu))
        return fail(ME_EINVAL, "invalid line data");
    me_line ln;
    std::memset(&ln, 0, sizeof ln);
    ln.lambda0_A = lambda0_A;
    double sum[3] = {0, 0, 0};
    int n = 0;
    for (int TM = -TJl; TM <= TJl; TM += 2) {
        for (int q = -1; q <= 1; ++q) {
            const int TMu = TM - 2 * q;
            if (TMu < -TJu || TMu > TJu)
                continue;
            const double s = cs_strength(TJl, TJu, TM, q);
            if (s <= 0.0)
                continue;
            if (n >= GENESIS_MAX_COMP)
                return fail(ME_EINVAL, "more than %d Zeeman components", GENESIS_MAX_COMP);
            ln.q[n] = q;
            ln.shift[n] = gl * 0.5 * TM - gu * 0.5 * TMu;
            ln.strength[n] = s;
            sum[q + 1] += s;
            ++n;
        }
    }
    for (int c = 0; c < n; ++c)
        ln.strength[c] /= sum[ln.q[c] + 1];
    ln.ncomp = n;
    *out = ln;
    return ME_OK;
}

int me_line_triplet(double lambda0_A, double geff, me_line *out)
{
    if (!out)
        return fail(ME_EINVAL, "out must not be NULL");
    if (!(lambda0_A > 0) || !std::isfinite(geff))
        return fail(ME_EINVAL, "invalid line data");
    me_line ln;
    std::memset(&ln, 0, sizeof ln);
    ln.lambda0_A = lambda0_A;
    ln.ncomp = 3;
    for (int c = 0; c < 3; ++c) {
        ln.q[c] = c - 1;
        ln.shift[c] = (c - 1) * geff;
        ln.strength[c] = 1.0;
    }
    *out = ln;
    return ME_OK;
}

int me_synth(const float *params, int64_t n, const me_line *lines, const me_grid *grids,
             int32_t nlines, const float *mu, float *stokes, void *stream)
{
    return synth_impl<float>(params, n, lines, grids, nlines, mu, stokes, stream);
}

int me_synth_f16(const float *params, int64_t n, const me_line *lines, const me_grid *grids,
                 int32_t nlines, const float *mu, float *stokes, void *stream)
{
    DevLines<float> ls;
    if (int rc = pack_lines(lines, grids, nlines, ls))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!params || !stokes)
        return fail(ME_EINVAL, "params and stokes must not be NULL");
    const int bs = 256;
    const int64_t blocks = (n + bs - 1) / bs;
    if (blocks > kMaxGrid)
        return fail(ME_EINVAL, "n too large");
    DevLinesH lh;
    pack_lines_h(ls, lh);
    hipLaunchKernelGGL(k_me_synth_h, dim3((unsigned)blocks), dim3(bs), 0, as_stream(stream),
                       params, n, ls, lh, mu, stokes);
    return check_launch("me_synth_f16");
}

int me_synth_f64(const double *params, int64_t n, const me_line *lines, const me_grid *grids,
                 int32_t nlines, const double *mu, double *stokes, void *stream)
{
    return synth_impl<double>(params, n, lines, grids, nlines, mu, stokes, stream);
}

int me_chi2(const float *params, int64_t npix, int32_t pop, const float *obs, const float *sigma,
            const float *mu, const me_line *lines, const me_grid *grids, int32_t nlines,
            float *chi2, void *stream)
{
    return fitness_impl<float, false>(params, nullptr, nullptr, npix, pop, obs, sigma, mu, lines,
                                      grids, nlines, chi2, stream);
}

int me_chi2_f64(const double *params, int64_t npix, int32_t pop, const double *obs,
                const double *sigma, const double *mu, const me_line *lines,
                const me_grid *grids, int32_t nlines, double *chi2, void *stream)
{
    return fitness_impl<double, false>(params, nullptr, nullptr, npix, pop, obs, sigma, mu, lines,
                                       grids, nlines, chi2, stream);
}

int ga_init(int64_t npix, const ga_config *cfg, const me_bounds *bounds, uint16_t *genes,
            void *stream)
{
    GaConst ga;
    if (int rc = pack_ga(cfg, ga))
        return rc;
    Bounds b{};
    if (ga.n_seeded > 0)
        if (int rc = pack_bounds(bounds, b))
            return rc;
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!genes)
        return fail(ME_EINVAL, "genes must not be NULL");
    const int64_t n = npix * cfg->pop;
    const int bs = 256;
    const int64_t blocks = (n + bs - 1) / bs;
    if (blocks > kMaxGrid)
        return fail(ME_EINVAL, "npix * pop too large");
    hipLaunchKernelGGL(k_ga_init, dim3((unsigned)blocks), dim3(bs), 0, as_stream(stream), npix,
                       ga, b, genes);
    return check_launch("ga_init");
}

int ga_restart(const uint16_t *genes_in, const float *fitness, int64_t npix,
               const ga_config *cfg, int32_t generation, uint16_t *genes_out, void *stream)
{
    return restart_impl<float>(genes_in, fitness, npix, cfg, generation, genes_out, stream);
}

int ga_restart_f64(const uint16_t *genes_in, const double *fitness, int64_t npix,
                   const ga_config *cfg, int32_t generation, uint16_t *genes_out, void *stream)
{
    return restart_impl<double>(genes_in, fitness, npix, cfg, generation, genes_out, stream);
}

int ga_decode(const uint16_t *genes, int64_t n, const me_bounds *bounds, float *params,
              void *stream)
{
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!genes || !params)
        return fail(ME_EINVAL, "NULL array argument");
    const int bs = 256;
    const int64_t blocks = (n + bs - 1) / bs;
    if (blocks > kMaxGrid)
        return fail(ME_EINVAL, "n too large");
    hipLaunchKernelGGL(k_decode<float>, dim3((unsigned)blocks), dim3(bs), 0, as_stream(stream),
                       genes, n, b, params);
    return check_launch("ga_decode");
}

int ga_evaluate(const uint16_t *genes, int64_t npix, int32_t pop, const me_bounds *bounds,
                const float *obs, const float *sigma, const float *mu, const me_line *lines,
                const me_grid *grids, int32_t nlines, float *fitness, void *stream)
{
    return fitness_impl<float, true>(nullptr, genes, bounds, npix, pop, obs, sigma, mu, lines,
                                     grids, nlines, fitness, stream);
}

int ga_evaluate_f64(const uint16_t *genes, int64_t npix, int32_t pop, const me_bounds *bounds,
                    const double *obs, const double *sigma, const double *mu,
                    const me_line *lines, const me_grid *grids, int32_t nlines,
                    double *fitness, void *stream)
{
    return fitness_impl<double, true>(nullptr, genes, bounds, npix, pop, obs, sigma, mu, lines,
                                      grids, nlines, fitness, stream);
}

int ga_step(const uint16_t *genes_in, const float *fitness, int64_t npix, const ga_config *cfg,
            int32_t generation, uint16_t *genes_out, int32_t *parents, int32_t *xpoint,
            uint16_t *masks, int32_t *elite, void *stream)
{
    return step_impl<float>(genes_in, fitness, npix, cfg, generation, genes_out, parents, xpoint,
                            masks, elite, stream);
}

int ga_step_f64(const uint16_t *genes_in, const double *fitness, int64_t npix,
                const ga_config *cfg, int32_t generation, uint16_t *genes_out, int32_t *parents,
                int32_t *xpoint, uint16_t *masks, int32_t *elite, void *stream)
{
    return step_impl<double>(genes_in, fitness, npix, cfg, generation, genes_out, parents, xpoint,
                             masks, elite, stream);
}

size_t ga_workspace_bytes(int64_t npix, const ga_config *cfg)
{
    (void)npix;
    (void)cfg;
    return 0;
}

int ga_invert_fill(const float *obs, const float *sigma, const float *mu, int64_t npix,
                   const me_line *lines, const me_grid *grids, int32_t nlines,
                   const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                   float *best_params, float *best_alpha, float *best_chi2, int32_t *status,
                   uint16_t *final_genes, float *final_fitness, void *stream)
{
    if (cfg && cfg->synth_precision == GENESIS_SYNTH_FP16)
        return invert_impl<float, GENESIS_SYNTH_FP16, true>(
            obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg, best_params, best_chi2,
            status, final_genes, final_fitness, stream, fill, best_alpha);
    if (cfg && cfg->synth_precision != GENESIS_SYNTH_NATIVE)
        return fail(ME_EINVAL, "synth_precision = %d is not a GENESIS_SYNTH_* value",
                    cfg->synth_precision);
    return invert_impl<float, GENESIS_SYNTH_NATIVE, true>(
        obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg, best_params, best_chi2, status,
        final_genes, final_fitness, stream, fill, best_alpha);
}

int ga_invert_fill_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const ga_config *cfg, const me_fill *fill,
                       double *best_params, double *best_alpha, double *best_chi2,
                       int32_t *status, uint16_t *final_genes, double *final_fitness,
                       void *stream)
{
    if (cfg && cfg->synth_precision != GENESIS_SYNTH_NATIVE)
        return fail(ME_EINVAL, "FP16 synthesis is an option of the FP32 search");
    return invert_impl<double, GENESIS_SYNTH_NATIVE, true>(
        obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg, best_params, best_chi2, status,
        final_genes, final_fitness, stream, fill, best_alpha);
}

int me_synth_fill(const float *params, const float *alpha, int64_t n, const me_line *lines,
                  const me_grid *grids, int32_t nlines, const float *mu, const me_fill *fill,
                  float *stokes, void *stream)
{
    return synth_fill_impl<float>(params, alpha, n, lines, grids, nlines, mu, fill, stokes,
                                  stream);
}

int me_synth_fill_f64(const double *params, const double *alpha, int64_t n,
                      const me_line *lines, const me_grid *grids, int32_t nlines,
                      const double *mu, const me_fill *fill, double *stokes, void *stream)
{
    return synth_fill_impl<double>(params, alpha, n, lines, grids, nlines, mu, fill, stokes,
                                   stream);
}

int ga_invert(const float *obs, const float *sigma, const float *mu, int64_t npix,
              const me_line *lines, const me_grid *grids, int32_t nlines,
              const me_bounds *bounds, const ga_config *cfg, float *best_params,
              float *best_chi2, int32_t *status, uint16_t *final_genes, float *final_fitness,
              void *workspace, size_t ws_bytes, void *stream)
{
    (void)workspace;
    (void)ws_bytes;
    return invert_dispatch<float>(obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg,
                              best_params, best_chi2, status, final_genes, final_fitness, stream);
}

int ga_invert_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const ga_config *cfg, double *best_params,
                  double *best_chi2, int32_t *status, uint16_t *final_genes,
                  double *final_fitness, void *workspace, size_t ws_bytes, void *stream)
{
    (void)workspace;
    (void)ws_bytes;
    return invert_dispatch<double>(obs, sigma, mu, npix, lines, grids, nlines, bounds, cfg,
                               best_params, best_chi2, status, final_genes, final_fitness,
                               stream);
}

int me_search_box(const double *obs, const double *sigma, int64_t npix, const me_line *lines,
                  const me_grid *grids, int32_t nlines, const me_bounds *bounds,
                  const double *prefit, double polarity_nsigma, float *box, void *stream)
{
    BoxArgs a{};
    if (int rc = pack_lines(lines, grids, nlines, a.ls))
        return rc;
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        a.lo[j] = bounds->lo[j];
        a.hi[j] = bounds->hi[j];
    }
    if (!std::isfinite(polarity_nsigma))
        return fail(ME_EINVAL, "polarity_nsigma must be finite");
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!box || (polarity_nsigma > 0.0 && (!obs || !sigma)))
        return fail(ME_EINVAL, "NULL array argument");
    a.obs = obs;
    a.sigma = sigma;
    a.prefit = prefit;
    a.npix = npix;
    a.nsigma = polarity_nsigma;
    a.box = box;
    hipLaunchKernelGGL(k_search_box, dim3(grid_for(npix)), dim3(kGuessThreads), 0,
                       as_stream(stream), a);
    return check_launch("me_search_box");
}

int me_invmax_sigma(const float *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                    double floor, float *sigma, void *stream)
{
    return invmax_impl(obs, npix, grids, nlines, floor, sigma, stream);
}

int me_invmax_sigma_f64(const double *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                        double floor, double *sigma, void *stream)
{
    return invmax_impl(obs, npix, grids, nlines, floor, sigma, stream);
}

int me_seeds(const double *obs, const double *mu, int64_t npix, const me_line *lines,
             const me_grid *grids, int32_t nlines, const me_bounds *bounds,
             const float *pixel_bounds, float *seeds, void *stream)
{
    SeedArgs sa{};
    if (int rc = pack_guess(obs, mu, npix, lines, grids, nlines, bounds, sa.g))
        return rc;
    if (npix == 0)
        return ME_OK;
    if (!obs || !seeds)
        return fail(ME_EINVAL, "NULL array argument");
    sa.box = pixel_bounds;
    sa.seeds = seeds;
    hipLaunchKernelGGL(k_seeds, dim3(grid_for(npix)), dim3(kGuessThreads), 0, as_stream(stream),
                       sa);
    return check_launch("me_seeds");
}

int me_first_guess(const double *obs, const double *mu, int64_t npix, const me_line *lines,
                   const me_grid *grids, int32_t nlines, const me_bounds *bounds, float *params,
                   void *stream)
{
    GuessArgs a{};
    if (int rc = pack_guess(obs, mu, npix, lines, grids, nlines, bounds, a))
        return rc;
    if (npix == 0)
        return ME_OK;
    if (!obs || !params)
        return fail(ME_EINVAL, "NULL array argument");
    a.params = params;
    hipLaunchKernelGGL(k_first_guess, dim3(grid_for(npix)), dim3(kGuessThreads), 0,
                       as_stream(stream), a);
    return check_launch("me_first_guess");
}

int me_refine_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const double *params_in, int32_t iterations,
                  double *params_out, double *chi2_out, int32_t *iters_done, void *stream)
{
    return refine_impl<false>(obs, sigma, mu, npix, lines, grids, nlines, bounds, params_in,
                              iterations, params_out, chi2_out, iters_done, stream);
}

int me_refine_fill_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                       const me_line *lines, const me_grid *grids, int32_t nlines,
                       const me_bounds *bounds, const me_fill *fill, const double *params_in,
                       const double *alpha_in, int32_t iterations, uint32_t free_mask,
                       double *params_out, double *alpha_out, double *chi2_out,
                       int32_t *iters_done, void *stream)
{
    return refine_impl<true>(obs, sigma, mu, npix, lines, grids, nlines, bounds, params_in,
                             iterations, params_out, chi2_out, iters_done, stream, free_mask,
                             false, fill, alpha_in, alpha_out);
}

int me_prefit_f64(const double *obs, const double *sigma, const double *mu, int64_t npix,
                  const me_line *lines, const me_grid *grids, int32_t nlines,
                  const me_bounds *bounds, const double *params_in, int32_t iterations,
                  double *params_out, double *chi2_out, int32_t *iters_done, void *stream)
{
    if (bounds && !(bounds->lo[0] <= 0.0 && bounds->hi[0] >= 0.0))
        return fail(ME_EINVAL, "the non-magnetic pre-fit needs a box containing B = 0");
    // v_los, Doppler width, damping, eta0, S0, S1 free; B held at 0 (the angles
    // then do not enter the model)
    return refine_impl<false>(obs, sigma, mu, npix, lines, grids, nlines, bounds, params_in,
                              iterations, params_out, chi2_out, iters_done, stream, 0x1f8u, true);
}

}  // extern "C"
