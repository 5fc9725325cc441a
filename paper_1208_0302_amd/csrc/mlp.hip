// Learned proposal: a multilayer perceptron that maps an observed Stokes
// vector to a first guess of the nine model parameters, used to seed part of
// the genetic algorithm's initial population (the paper seeds its population
// with heuristic first guesses, Sec. 5.5, and cites neural-network inversion,
// Sec. 1).  Architecture: 1024 inputs (4 Stokes x 256 samples, normalised by
// the pixel's maximum of I) -> 3 x 512 GELU -> 9 outputs (parameters scaled
// to [0, 1] by the search box).
//
// Matrix products run on the MFMA units: BF16 operands, FP32 accumulation
// (v_mfma_f32_32x32x16_bf16), FP32 master weights with Adam.  An FP32 mode
// (VALU FMA tiles) exists for gradient checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "genesis_common.h"

namespace {

using namespace genesis;

constexpr int kIn = 1024, kHid = 512, kOut = 9, kLayers = 4;
constexpr int kDims[kLayers + 1] = {kIn, kHid, kHid, kHid, kOut};

// parameter offsets: W_l [out][in] then b_l [out], layer by layer
constexpr int64_t w_off(int l)
{
    int64_t o = 0;
    for (int i = 0; i < l; ++i)
        o += (int64_t)kDims[i + 1] * kDims[i] + kDims[i + 1];
    return o;
}
constexpr int64_t b_off(int l) { return w_off(l) + (int64_t)kDims[l + 1] * kDims[l]; }
constexpr int64_t kParams = w_off(kLayers);

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (values here are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ T to_store(float x);
template <>
__device__ __forceinline__ uint16_t to_store<uint16_t>(float x) { return f2bf(x); }
template <>
__device__ __forceinline__ float to_store<float>(float x) { return x; }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum Epi : int { kFwdHidden = 0, kFwdOut = 1, kBwdHidden = 2, kGradW = 3, kBwdPlain = 4 };

struct GemmArgs {
    const void *A, *B;  // element type T
    int M, N, K;
    int lda, ldb;       // leading dimensions of A, B as stored
    const float *bias;  // [N]            (forward)
    const float *pre_in;  // [M][N]       (backward: pre-activation)
    float *outf;        // [M][N] f32 result (pre-activation / output / gradient)
    void *outt;         // [M][N] T result (activation or gradient operand)
    // split-K weight gradients (bf16 path): block z covers k in [z kper, (z + 1) kper)
    // and writes its partial product to outf + z M N; block (x, y, z) also sums
    // bsrc[k][m] (f32 [K][M]) over the x-th of gridDim.x equal slices of that k
    // range into bpart[z gridDim.x + x][m] (the bias-gradient partials)
    int kper;
    const float *bsrc;
    float *bpart;
};

// Epilogue of one accumulated element (m, n).
template <typename T, int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs &a, int m, int n, float acc)
{
    if (m >= a.M || n >= a.N)
        return;
    const int64_t i = (int64_t)m * a.N + n;
    if (EPI == kFwdHidden) {
        const float pre = acc + a.bias[n];
        a.outf[i] = pre;
        ((T *)a.outt)[i] = to_store<T>(gelu(pre));
    } else if (EPI == kFwdOut) {
        a.outf[i] = acc + a.bias[n];
    } else if (EPI == kBwdHidden) {
        const float d = acc * gelu_d(a.pre_in[i]);
        a.outf[i] = d;
        ((T *)a.outt)[i] = to_store<T>(d);
    } else {  // kGradW, kBwdPlain
        a.outf[i] = acc;
    }
}

// One 64 x 64 bf16 tile of a matrix operand, element (r, c) = global
// (row0 + r, k0 + c), moved global -> registers -> LDS T[r][c] (k contiguous
// in LDS), in chunks of 8 elements contiguous in memory.  EDGE = false: the
// chunks are 16-byte aligned and each lies wholly inside or wholly outside the
// matrix (leading dimension, base and the chunked extent multiples of 8), so a
// chunk is one unconditional 16-byte load (from the base when outside, then
// zeroed): no branches, which lets loads of later k-steps stay in flight.
// EDGE = true: element loads with zero fill where a chunk is not whole.
constexpr int kTile = 64, kTileK = 64, kLdsPitch = kTileK + 8;

// EDGE = false returns the raw load; the caller zeroes it (keep) when it is
// consumed, so that the load is not waited for here.
template <bool EDGE>
__device__ __forceinline__ bf16x8 load8(const uint16_t *__restrict__ X, int64_t base, bool whole,
                                        int nvalid)
{
    if (!EDGE)
        return *(const bf16x8 *)(X + (whole ? base : 0));
    if (whole && ((uintptr_t)(X + base) & 15) == 0)
        return *(const bf16x8 *)(X + base);
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        v[e] = e < nvalid ? (short)X[base + e] : (short)0;
    return v;
}

template <bool KC, bool EDGE>
struct TileLoader;

__device__ __forceinline__ bf16x8 keep(bf16x8 v, bool whole)
{
    const bf16x8 z = {0};
    return whole ? v : z;
}

// Stored with k contiguous ([rows][ld]): each of the 256 threads owns two
// chunks of 8 consecutive k of one row, written to LDS as 16 bytes (8 lanes
// fill one 128-byte LDS row segment: conflict-free).
template <bool EDGE>
struct TileLoader<true, EDGE> {
    bf16x8 v[2];
    bool whole[2];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ X, int ld, int rows, int K,
                                         int row0, int k0, int tid)
    {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = tid + 256 * j;
            const int gr = row0 + (q >> 3), gc = k0 + (q & 7) * 8;
            const bool in_row = gr < rows;
            whole[j] = in_row && gc + 8 <= K && (EDGE ? (ld & 7) == 0 : true);
            v[j] = load8<EDGE>(X, (int64_t)gr * ld + gc, whole[j], in_row ? min(8, K - gc) : 0);
        }
    }

    __device__ __forceinline__ void store(uint16_t (*T)[kLdsPitch], int tid) const
    {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = tid + 256 * j;
            *(bf16x8 *)&T[q >> 3][(q & 7) * 8] = EDGE ? v[j] : keep(v[j], whole[j]);
        }
    }
};

// Stored with rows contiguous ([K][ld]): thread t loads rows 8 (t / 32) ..
// + 7 of the two k-columns 2 (t % 32) and 2 (t % 32) + 1 (two 16-byte loads),
// pairs the two k of each row into one dword and writes 8 dwords; the 32
// lanes of a half-wave write 128 consecutive bytes of one LDS row, so the
// transposing store is conflict-free.
template <bool EDGE>
struct TileLoader<false, EDGE> {
    bf16x8 v[2];
    bool whole[2];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ X, int ld, int rows, int K,
                                         int row0, int k0, int tid)
    {
        const int gr = row0 + 8 * (tid >> 5);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int gc = k0 + 2 * (tid & 31) + j;
            const bool in_k = gc < K;
            whole[j] = in_k && gr + 8 <= rows && (EDGE ? (ld & 7) == 0 : true);
            v[j] = load8<EDGE>(X, (int64_t)gc * ld + gr, whole[j], in_k ? min(8, rows - gr) : 0);
        }
    }

    __device__ __forceinline__ void store(uint16_t (*T)[kLdsPitch], int tid) const
    {
        const int r = 8 * (tid >> 5), c = 2 * (tid & 31);
        const bf16x8 v0 = EDGE ? v[0] : keep(v[0], whole[0]);
        const bf16x8 v1 = EDGE ? v[1] : keep(v[1], whole[1]);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t w = (uint32_t)(uint16_t)v0[e] | ((uint32_t)(uint16_t)v1[e] << 16);
            *(uint32_t *)&T[r + e][c] = w;
        }
    }
};

// One k-step of a tile product: registers -> LDS buffer, one barrier, the
// loads of the step two ahead into the same registers, then the four MFMAs of
// each wave.  The two LDS buffers alternate with the two register stages, so
// the store of the next step never overwrites a buffer still being read and
// one barrier per step suffices.
template <bool TA, bool TB, bool EDGE>
__device__ __forceinline__ void gemm_step(TileLoader<!TA, EDGE> &la, TileLoader<TB, EDGE> &lb,
                                          uint16_t (*As)[kLdsPitch], uint16_t (*Bs)[kLdsPitch],
                                          const GemmArgs &a, int ke, int m0, int n0, int knext,
                                          int tid, int lane, int wm, int wn, f32x16 &acc)
{
    la.store(As, tid);
    lb.store(Bs, tid);
    __syncthreads();
    // whole-chunk loaders load unconditionally (past ke every chunk reads the
    // operand base and is zeroed), so the number of loads in flight is the
    // same on every path and each store waits only for its own step's loads
    if (!EDGE || knext < ke) {
        la.load((const uint16_t *)a.A, a.lda, a.M, ke, m0, knext, tid);
        lb.load((const uint16_t *)a.B, a.ldb, a.N, ke, n0, knext, tid);
    }
#pragma unroll
    for (int kk = 0; kk < kTileK; kk += 16) {
        const int kr = kk + 8 * (lane >> 5);
        const bf16x8 av = *(const bf16x8 *)&As[wm + (lane & 31)][kr];
        const bf16x8 bv = *(const bf16x8 *)&Bs[wn + (lane & 31)][kr];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
}

// C[M][N] = op(A)[M][K] op(B)[K][N].  TA: A stored [K][M]; TB: B stored [N][K].
// Block 256 threads (4 waves in 2 x 2, each a 32 x 32 MFMA tile), 64 x 64
// output tile, k step 64 staged through two LDS buffers, with the operands of
// the next two steps in flight in registers.
template <bool TA, bool TB, int EPI, bool EDGE>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs a)
{
    __shared__ __align__(16) uint16_t As[2][kTile][kLdsPitch];
    __shared__ __align__(16) uint16_t Bs[2][kTile][kLdsPitch];
    const uint16_t *A = (const uint16_t *)a.A, *B = (const uint16_t *)a.B;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const bool split = EPI == kGradW;
    const int kb = split ? blockIdx.z * a.kper : 0;
    const int ke = split ? min(a.K, kb + a.kper) : a.K;
    TileLoader<!TA, EDGE> la0, la1;
    TileLoader<TB, EDGE> lb0, lb1;
    la0.load(A, a.lda, a.M, ke, m0, kb, tid);
    lb0.load(B, a.ldb, a.N, ke, n0, kb, tid);
    la1.load(A, a.lda, a.M, ke, m0, kb + kTileK, tid);
    lb1.load(B, a.ldb, a.N, ke, n0, kb + kTileK, tid);
    f32x16 acc = {0};
    const int nsteps = ke > kb ? (ke - kb + kTileK - 1) / kTileK : 0;
    int st = 0;
    for (; st + 2 <= nsteps; st += 2) {
        const int k0 = kb + st * kTileK;
        gemm_step<TA, TB, EDGE>(la0, lb0, As[0], Bs[0], a, ke, m0, n0, k0 + 2 * kTileK, tid, lane,
                                wm, wn, acc);
        gemm_step<TA, TB, EDGE>(la1, lb1, As[1], Bs[1], a, ke, m0, n0, k0 + 3 * kTileK, tid, lane,
                                wm, wn, acc);
    }
    if (st < nsteps)
        gemm_step<TA, TB, EDGE>(la0, lb0, As[0], Bs[0], a, ke, m0, n0, ke, tid, lane, wm, wn, acc);
    // D layout: column n = lane % 32, row m = 8 (r / 4) + 4 (lane / 32) + r % 4
    GemmArgs e = a;
    if (split)
        e.outf = a.outf + (int64_t)blockIdx.z * a.M * a.N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn + (lane & 31);
        epilogue<uint16_t, EPI>(e, m, n, acc[r]);
    }
    if (split) {
        // bias-gradient partial of rows m0 .. m0 + 63 over this block's slice
        // of the k range: thread (c, r) sums k = k1 + r, k1 + r + 4, ... in
        // order, then the four phases are added in order
        const int sub = (ke - kb + gridDim.x - 1) / gridDim.x;
        const int k1 = kb + blockIdx.x * sub, k2 = min(ke, k1 + sub);
        __syncthreads();  // the last step's MFMA operands may still be read
        float(*part)[64] = (float(*)[64])&As[0][0][0];
        const int c = tid & 63, ph = tid >> 6, m = m0 + c;
        float s = 0.0f;
        if (m < a.M) {
#pragma unroll 4
            for (int k = k1 + ph; k < k2; k += 4)
                s += a.bsrc[(int64_t)k * a.M + m];
        }
        part[ph][c] = s;
        __syncthreads();
        if (ph == 0 && m < a.M)
            a.bpart[((int64_t)blockIdx.z * gridDim.x + blockIdx.x) * a.M + m] =
                ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
    }
}

// Sum of the split-K partials in block order: out[i] = sum_z part[z][i] for the
// weight gradient (n elements) and bout[m] = sum_q bpart[q][m] over the P bias
// partials (nb elements).
__global__ __launch_bounds__(256) void k_split_sum(const float *__restrict__ part, int S, int64_t n,
                                                   float *__restrict__ out,
                                                   const float *__restrict__ bpart, int P, int nb,
                                                   float *__restrict__ bout)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((n & 3) == 0 && 4 * i + 3 < n) {
        float4 s = ((const float4 *)part)[i];
        for (int z = 1; z < S; ++z) {
            const float4 t = ((const float4 *)(part + z * n))[i];
            s.x += t.x;
            s.y += t.y;
            s.z += t.z;
            s.w += t.w;
        }
        ((float4 *)out)[i] = s;
    } else if ((n & 3) != 0) {
        for (int64_t j = 4 * i; j < min(4 * i + 4, n); ++j) {
            float s = part[j];
            for (int z = 1; z < S; ++z)
                s += part[z * n + j];
            out[j] = s;
        }
    }
    if (i < nb) {
        // in order; the unrolled loads are all in flight before the adds
        float s = bpart[i];
#pragma unroll 16
        for (int q = 1; q < P; ++q)
            s += bpart[q * nb + i];
        bout[i] = s;
    }
}

// FP32 reference-precision product on the VALU (gradient checks).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs a)
{
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ float As[BK][BM + 1];
    __shared__ float Bs[BK][BN + 1];
    const float *A = (const float *)a.A, *B = (const float *)a.B;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int tid = threadIdx.x;
    const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < a.K; k0 += BK) {
        for (int e = tid; e < BM * BK; e += 256) {
            const int c = e / BM, r = e % BM;
            const int gm = m0 + r, gk = k0 + c;
            As[c][r] = (gm < a.M && gk < a.K)
                           ? (TA ? A[(int64_t)gk * a.lda + gm] : A[(int64_t)gm * a.lda + gk])
                           : 0.0f;
        }
        for (int e = tid; e < BN * BK; e += 256) {
            const int c = e / BN, r = e % BN;
            const int gn = n0 + r, gk = k0 + c;
            Bs[c][r] = (gn < a.N && gk < a.K)
                           ? (TB ? B[(int64_t)gn * a.ldb + gk] : B[(int64_t)gk * a.ldb + gn])
                           : 0.0f;
        }
        __syncthreads();
        for (int k = 0; k < BK; ++k)
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = fmaf(As[k][tm + i], Bs[k][tn + j], acc[i][j]);
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            epilogue<float, EPI>(a, m0 + tm + i, n0 + tn + j, acc[i][j]);
}

// column sums: out[n] = sum_m in[m][n].  Block (64 columns) x (16 row
// phases); thread (c, r) sums rows r, r + 16, ... in order, then the 16
// partials are added in order: a fixed summation order for every launch.
__global__ __launch_bounds__(1024) void k_colsum(const float *in, int M, int N, float *out)
{
    __shared__ float part[16][64];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float s = 0.0f;
    if (n < N)
        for (int m = r; m < M; m += 16)
            s += in[(int64_t)m * N + n];
    part[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N) {
        float t = 0.0f;
        for (int i = 0; i < 16; ++i)
            t += part[i][c];
        out[n] = t;
    }
}

template <typename T>
__global__ void k_cast(const float *in, int64_t n, T *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = to_store<T>(in[i]);
}

// Loss: mean over the batch of sum_j d_j^2 with d = out - target, the azimuth
// (j = 2) taken modulo 1 (its 180-degree period).  Writes dL/dout (f32 and T)
// and the per-sample loss.
template <typename T>
__global__ void k_loss(const float *out, const float *target, int B, float *dout_f, T *dout_t,
                       float *per_sample)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    float s = 0.0f;
    for (int j = 0; j < kOut; ++j) {
        float d = out[b * kOut + j] - target[b * kOut + j];
        if (j == 2)
            d = d - rintf(d);
        s = fmaf(d, d, s);
        const float g = 2.0f * d / (float)B;
        dout_f[b * kOut + j] = g;
        dout_t[b * kOut + j] = to_store<T>(g);
    }
    per_sample[b] = s;
}

// out = scale * sum in[0..n): 256 strided partial sums, then a fixed tree.
__global__ __launch_bounds__(256) void k_sum(const float *in, int n, float scale, float *out)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256)
        s += in[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = red[0] * scale;
}

__global__ void k_adam(float *p, float *m, float *v, const float *g, int64_t n, float lr,
                       float b1, float omb1, float b2, float omb2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], omb1 * gi);
    const float vi = fmaf(b2, v[i], omb2 * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// He-normal weights (Box-Muller on Philox words), zero biases.
__global__ void k_init(float *p, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams)
        return;
    int l = 0;
    while (l + 1 < kLayers && i >= w_off(l + 1))
        ++l;
    if (i >= b_off(l)) {
        p[i] = 0.0f;
        return;
    }
    const Key key{(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint4 w = philox((uint32_t)i, (uint32_t)(i >> 32), 0u, 6u << 24, key);
    const float u1 = ((w.x >> 8) + 1) * (1.0f / 16777217.0f), u2 = (w.y >> 8) * (1.0f / 16777216.0f);
    const float z = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
    p[i] = z * sqrtf(2.0f / (float)kDims[l]);
}

// features: x[p][s*L + j] = obs[p][s][j] / max_j obs[p][0][j]
__global__ void k_features(const float *obs, int64_t npix, int L, float *x)
{
    const int64_t p = blockIdx.x;
    if (p >= npix)
        return;
    __shared__ float red[256];
    float mx = -INFINITY;
    for (int j = threadIdx.x; j < L; j += blockDim.x)
        mx = fmaxf(mx, obs[p * 4 * L + j]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = (int)blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float inv = 1.0f / red[0];
    for (int e = threadIdx.x; e < 4 * L; e += blockDim.x)
        x[p * 4 * L + e] = obs[p * 4 * L + e] * inv;
}

// Training examples drawn on the device: parameters uniform in the box
// (v_los normal, sigma = box width / 10, clipped), and the scaled targets.
__global__ void k_draw(uint64_t seed, int64_t first, int64_t n, Bounds b, float *params,
                       float *target)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t gi = first + i;
    const Key key{(uint32_t)seed, (uint32_t)(seed >> 32)};
    const uint4 w0 = philox((uint32_t)gi, (uint32_t)(gi >> 32), 1u, 7u << 24, key);
    const uint4 w1 = philox((uint32_t)gi, (uint32_t)(gi >> 32), 1u, (7u << 24) | 1u, key);
    const uint4 w2 = philox((uint32_t)gi, (uint32_t)(gi >> 32), 1u, (7u << 24) | 2u, key);
    const uint32_t ws[12] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w, w2.x, w2.y, w2.z, w2.w};
    for (int j = 0; j < GENESIS_NPAR; ++j) {
        float u = (ws[j] >> 8) * (1.0f / 16777216.0f);
        if (j == 3) {  // normal around the box centre, sigma = width / 10
            const float u1 = ((ws[9] >> 8) + 1) * (1.0f / 16777217.0f);
            const float u2 = (ws[10] >> 8) * (1.0f / 16777216.0f);
            const float z = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
            u = fminf(fmaxf(0.5f + 0.1f * z, 0.0f), 1.0f);
        }
        params[i * GENESIS_NPAR + j] = (float)(b.lo[j] + b.span[j] * u);
        target[i * GENESIS_NPAR + j] = u;
    }
}

// additive Gaussian noise sigma_rel * (S0 + S1) on every sample (mu = 1)
__global__ void k_noise(uint64_t seed, int64_t first, const float *params, int64_t n, int L,
                        float sigma_rel, float *stokes)
{
    const int64_t p = blockIdx.x;
    if (p >= n)
        return;
    const float ic = params[p * GENESIS_NPAR + 7] + params[p * GENESIS_NPAR + 8];
    const Key key{(uint32_t)seed, (uint32_t)(seed >> 32)};
    const int64_t gp = first + p;
    for (int e = threadIdx.x; e < 4 * L; e += blockDim.x) {
        const uint4 w = philox((uint32_t)gp, (uint32_t)(gp >> 32), 2u, (8u << 24) | (uint32_t)e, key);
        const float u1 = ((w.x >> 8) + 1) * (1.0f / 16777217.0f), u2 = (w.y >> 8) * (1.0f / 16777216.0f);
        const float z = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        stokes[p * 4 * L + e] += sigma_rel * ic * z;
    }
}

// scaled outputs -> parameters inside the box
__global__ void k_unscale(const float *out, int64_t n, Bounds b, float *params)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * GENESIS_NPAR)
        return;
    const int j = (int)(i % GENESIS_NPAR);
    float u = out[i];
    if (j == 2)
        u = u - floorf(u);
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    params[i] = (float)(b.lo[j] + b.span[j] * u);
}

// ---- workspace ------------------------------------------------------------

struct Ws {
    uint16_t *wbf;             // bf16 weights [kParams]
    float *x;                  // input [B][1024] f32
    uint16_t *xb;              // input bf16
    float *pre[3];             // pre-activations [B][512]
    void *act[3];              // activations [B][512] (T)
    float *out;                // [B][9]
    float *dout_f;             // [B][9]
    void *dout_t;              // [B][9] (T)
    float *dh_f;               // [B][512]
    void *dh_t[2];             // [B][512] (T)
    float *per_sample;         // [B]
    float *split;              // split-K weight-gradient partials [kSplitMax][512 * 1024]
    float *bsplit;             // bias-gradient partials [kSplitMax * 16][512]
};

// Split-K factor of a weight-gradient product with `tiles` output tiles and
// K = batch: enough splits for about 512 workgroups, at least 128 k per split.
constexpr int kSplitMax = 8;
int split_of(int tiles, int64_t K)
{
    int s = (512 + tiles - 1) / tiles;
    s = (int)std::min<int64_t>(s, std::max<int64_t>(1, K / 128));
    return std::max(1, std::min(s, kSplitMax));
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ws_bytes(int64_t B)
{
    size_t s = 0;
    s += al(kParams * 2);
    s += al(B * kIn * 4) + al(B * kIn * 2);
    s += 3 * (al(B * kHid * 4) + al(B * kHid * 4));
    s += al(B * kOut * 4) * 2 + al(B * kOut * 4);
    s += al(B * kHid * 4) + 2 * al(B * kHid * 4);
    s += al(B * 4);
    s += al((size_t)kSplitMax * kHid * kIn * 4) + al((size_t)kSplitMax * (kIn / 64) * kHid * 4);
    return s;
}

Ws ws_layout(void *base, int64_t B)
{
    char *p = (char *)base;
    Ws w;
    auto take = [&](size_t n) {
        char *r = p;
        p += al(n);
        return (void *)r;
    };
    w.wbf = (uint16_t *)take(kParams * 2);
    w.x = (float *)take(B * kIn * 4);
    w.xb = (uint16_t *)take(B * kIn * 2);
    for (int i = 0; i < 3; ++i) {
        w.pre[i] = (float *)take(B * kHid * 4);
        w.act[i] = take(B * kHid * 4);
    }
    w.out = (float *)take(B * kOut * 4);
    w.dout_f = (float *)take(B * kOut * 4);
    w.dout_t = take(B * kOut * 4);
    w.dh_f = (float *)take(B * kHid * 4);
    w.dh_t[0] = take(B * kHid * 4);
    w.dh_t[1] = take(B * kHid * 4);
    w.per_sample = (float *)take(B * 4);
    w.split = (float *)take((size_t)kSplitMax * kHid * kIn * 4);
    w.bsplit = (float *)take((size_t)kSplitMax * (kIn / 64) * kHid * 4);
    return w;
}

// The forward pass alone needs the BF16 weights, the input (FP32 and BF16),
// the three hidden layers (pre-activation and activation) and the output, in
// the same order as ws_layout places them.
size_t fwd_bytes(int64_t B)
{
    return al(kParams * 2) + al(B * kIn * 4) + al(B * kIn * 2) +
           3 * (al(B * kHid * 4) + al(B * kHid * 4)) + al(B * kOut * 4);
}

Ws fwd_layout(void *base, int64_t B)
{
    char *p = (char *)base;
    Ws w{};
    auto take = [&](size_t n) {
        char *r = p;
        p += al(n);
        return (void *)r;
    };
    w.wbf = (uint16_t *)take(kParams * 2);
    w.x = (float *)take(B * kIn * 4);
    w.xb = (uint16_t *)take(B * kIn * 2);
    for (int i = 0; i < 3; ++i) {
        w.pre[i] = (float *)take(B * kHid * 4);
        w.act[i] = take(B * kHid * 4);
    }
    w.out = (float *)take(B * kOut * 4);
    return w;
}

// Scratch of mlp_forward_noalloc: one forward workspace of kNoAllocRows rows
// per device, a file-scope device array.  Host code must not pass the array's
// name to a kernel (that is a host-side stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocRows = 1024;
constexpr size_t kNoAllocBytes = (kParams * 2 + 255) / 256 * 256 + kNoAllocRows * kIn * 4 +
                                 kNoAllocRows * kIn * 2 + 6 * kNoAllocRows * kHid * 4 +
                                 (kNoAllocRows * kOut * 4 + 255) / 256 * 256;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];
hipError_t g_scratch_rc[kMaxDevices];

// The scratch array's device address on the current device (set up once per
// device, with that device current).
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(ME_EHIP, "no current device (or device index >= %d)", kMaxDevices);
    std::call_once(g_scratch_once[dev], [dev] {
        g_scratch_rc[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_rc[dev] != hipSuccess || !g_scratch_ptr[dev])
        return fail(ME_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(g_scratch_rc[dev]));
    *out = g_scratch_ptr[dev];
    return ME_OK;
}

// training area after the pass workspace: drawn parameters, targets, the
// synthesised Stokes vectors and the gradient
struct TrainWs {
    float *params, *target, *stokes, *grad;
};

size_t train_ws_bytes(int64_t B, int L)
{
    return ws_bytes(B) + 2 * al(B * kOut * 4) + al(B * 4 * (int64_t)L * 4) + al(kParams * 4);
}

TrainWs train_layout(void *base, int64_t B, int L)
{
    char *p = (char *)base + ws_bytes(B);
    TrainWs t;
    t.params = (float *)p;
    p += al(B * kOut * 4);
    t.target = (float *)p;
    p += al(B * kOut * 4);
    t.stokes = (float *)p;
    p += al(B * 4 * (int64_t)L * 4);
    t.grad = (float *)p;
    return t;
}

// Whether every 8-element chunk the bf16 tile loaders read is 16-byte aligned
// and wholly inside or wholly outside its operand (the branch-free loaders).
bool whole_chunks(const GemmArgs &a, bool TA, bool TB)
{
    auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    // A: k-contiguous rows (chunks along K) unless TA (chunks along M)
    const bool okA = (a.lda & 7) == 0 && ((TA ? a.M : a.K) & 7) == 0 && al16(a.A);
    // B: k-contiguous rows when TB (chunks along K), else chunks along N
    const bool okB = (a.ldb & 7) == 0 && ((TB ? a.K : a.N) & 7) == 0 && al16(a.B);
    return okA && okB;
}

template <bool TA, bool TB, int EPI>
void launch_bf16(dim3 grid, const GemmArgs &a, hipStream_t st)
{
    if (whole_chunks(a, TA, TB))
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, false>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI, true>), grid, dim3(256), 0, st, a);
}

template <int EPI, bool TA, bool TB>
int gemm(bool bf16, GemmArgs a, hipStream_t st)
{
    const dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
    if (bf16)
        launch_bf16<TA, TB, EPI>(grid, a, st);
    else
        hipLaunchKernelGGL((k_gemm_f32<TA, TB, EPI>), grid, dim3(256), 0, st, a);
    return check_launch("mlp gemm");
}

int blocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

// forward pass from ws.x (f32 input); weights: bf16 copy in ws.wbf or the f32 masters
int forward(bool bf16, const float *master, const Ws &w, int64_t B, hipStream_t st)
{
    if (bf16) {
        hipLaunchKernelGGL(k_cast<uint16_t>, dim3(blocks(kParams, 256)), dim3(256), 0, st, master,
                           kParams, w.wbf);
        hipLaunchKernelGGL(k_cast<uint16_t>, dim3(blocks(B * kIn, 256)), dim3(256), 0, st, w.x,
                           B * kIn, w.xb);
    }
    const void *in = bf16 ? (const void *)w.xb : (const void *)w.x;
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs a{};
        a.A = in;
        a.B = bf16 ? (const void *)(w.wbf + w_off(l)) : (const void *)(master + w_off(l));
        a.M = (int)B;
        a.N = kDims[l + 1];
        a.K = kDims[l];
        a.lda = kDims[l];
        a.ldb = kDims[l];  // W stored [out][in] = B transposed
        a.bias = master + b_off(l);
        int rc;
        if (l < kLayers - 1) {
            a.outf = w.pre[l];
            a.outt = w.act[l];
            rc = gemm<kFwdHidden, false, true>(bf16, a, st);
            in = w.act[l];
        } else {
            a.outf = w.out;
            rc = gemm<kFwdOut, false, true>(bf16, a, st);
        }
        if (rc)
            return rc;
    }
    return ME_OK;
}

int backward(bool bf16, const float *master, const Ws &w, int64_t B, float *grad, hipStream_t st)
{
    // layer 3 (output): dW3 = dout^T act2, db3 = colsum(dout), dh = dout W3 * gelu'(pre2)
    const void *dcur = w.dout_t;
    const float *dcur_f = w.dout_f;
    int buf = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int nout = kDims[l + 1], nin = kDims[l];
        const void *act_in = l == 0 ? (bf16 ? (const void *)w.xb : (const void *)w.x)
                                    : w.act[l - 1];
        GemmArgs g{};
        g.A = dcur;  // dY [B][nout] used transposed: A[m = out][k = b]
        g.B = act_in;  // X [B][nin]: B[k = b][n = in]
        g.M = nout;
        g.N = nin;
        g.K = (int)B;
        g.lda = nout;
        g.ldb = nin;
        if (bf16) {
            // split K = batch over blockIdx.z, partials summed in block order
            const int tiles = ((nout + 63) / 64) * ((nin + 63) / 64);
            const int S = split_of(tiles, B);
            g.kper = (int)((((B + S - 1) / S) + kTileK - 1) / kTileK * kTileK);
            const int S_used = (int)((B + g.kper - 1) / g.kper);
            g.outf = w.split;
            g.bsrc = dcur_f;
            g.bpart = w.bsplit;
            const int nx = (nin + 63) / 64;  // <= kIn / 64
            launch_bf16<true, false, kGradW>(dim3(nx, (nout + 63) / 64, S_used), g, st);
            const int64_t n = (int64_t)nout * nin;
            hipLaunchKernelGGL(k_split_sum, dim3(blocks(std::max<int64_t>((n + 3) / 4, nout), 256)),
                               dim3(256), 0, st, (const float *)w.split, S_used, n,
                               grad + w_off(l), (const float *)w.bsplit, S_used * nx, nout,
                               grad + b_off(l));
            if (int rc = check_launch("mlp weight gradient"))
                return rc;
        } else {
            g.outf = grad + w_off(l);
            if (int rc = gemm<kGradW, true, false>(bf16, g, st))
                return rc;
            hipLaunchKernelGGL(k_colsum, dim3(blocks(nout, 64)), dim3(1024), 0, st, dcur_f,
                               (int)B, nout, grad + b_off(l));
        }
        if (l == 0)
            break;
        GemmArgs d{};
        d.A = dcur;  // dY [B][nout]
        d.B = bf16 ? (const void *)(w.wbf + w_off(l)) : (const void *)(master + w_off(l));
        d.M = (int)B;
        d.N = nin;
        d.K = nout;
        d.lda = nout;
        d.ldb = nin;  // W [out][in] = B[k = out][n = in] row-major
        d.pre_in = w.pre[l - 1];
        d.outf = w.dh_f;
        d.outt = w.dh_t[buf];
        if (int rc = gemm<kBwdHidden, false, false>(bf16, d, st))
            return rc;
        dcur = w.dh_t[buf];
        dcur_f = w.dh_f;
        buf ^= 1;
    }
    return check_launch("mlp backward");
}

}  // namespace

extern "C" {

int64_t mlp_param_count(void) { return kParams; }

size_t mlp_workspace_bytes(int64_t batch) { return batch > 0 ? ws_bytes(batch) : 0; }

int mlp_init(float *master, uint64_t seed, void *stream)
{
    if (!master)
        return fail(ME_EINVAL, "master must not be NULL");
    hipLaunchKernelGGL(k_init, dim3(blocks(kParams, 256)), dim3(256), 0, as_stream(stream),
                       master, seed);
    return check_launch("mlp_init");
}

int mlp_features(const float *obs, int64_t npix, const me_grid *grids, int32_t nlines,
                 float *x, void *stream)
{
    if (!grids || nlines < 1 || nlines > GENESIS_MAX_LINES)
        return fail(ME_EINVAL, "invalid grids");
    int L = 0;
    for (int i = 0; i < nlines; ++i)
        L += grids[i].n;
    if (4 * L != kIn)
        return fail(ME_EINVAL, "the network takes 4 L = %d inputs, got L = %d", kIn, L);
    if (npix < 0)
        return fail(ME_EINVAL, "npix must be >= 0");
    if (npix == 0)
        return ME_OK;
    if (!obs || !x)
        return fail(ME_EINVAL, "NULL array argument");
    hipLaunchKernelGGL(k_features, dim3((unsigned)npix), dim3(256), 0, as_stream(stream), obs,
                       npix, L, x);
    return check_launch("mlp_features");
}

int mlp_forward(const float *master, const float *x, int64_t n, int32_t precision, float *y,
                void *workspace, size_t ws, void *stream)
{
    if (!master || !x || !y || !workspace)
        return fail(ME_EINVAL, "NULL argument");
    if (n < 1 || ws < ws_bytes(n))
        return fail(ME_ENOMEM, "workspace of %zu B too small for %lld rows", ws, (long long)n);
    const bool bf16 = precision == 0;
    Ws w = ws_layout(workspace, n);
    hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(w.x, x, n * kIn * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    if (int rc = forward(bf16, master, w, n, st))
        return rc;
    if (hipMemcpyAsync(y, w.out, n * kOut * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    return ME_OK;
}

int64_t mlp_noalloc_max_rows(void) { return kNoAllocRows; }

int mlp_forward_noalloc(const float *master, const float *x, int64_t n, int32_t precision,
                        float *y, void *stream)
{
    if (!master || !x || !y)
        return fail(ME_EINVAL, "NULL argument");
    if (n < 1 || n > kNoAllocRows)
        return fail(ME_EINVAL, "mlp_forward_noalloc takes 1 to %lld rows per call, got %lld",
                    (long long)kNoAllocRows, (long long)n);
    void *base = nullptr;
    if (int rc = scratch_address(&base))
        return rc;
    if (fwd_bytes(n) > kNoAllocBytes)
        return fail(ME_ENOMEM, "internal: forward scratch of %zu B exceeds %zu B", fwd_bytes(n),
                    kNoAllocBytes);
    const bool bf16 = precision == 0;
    const Ws w = fwd_layout(base, n);
    hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(w.x, x, n * kIn * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    if (int rc = forward(bf16, master, w, n, st))
        return rc;
    if (hipMemcpyAsync(y, w.out, n * kOut * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    return ME_OK;
}

}  // extern "C"

namespace {

// loss and gradient of one batch whose features are already in w.x
int grad_pass(bool bf16, const float *master, const Ws &w, const float *target, int64_t batch,
              float *grad, float *loss, hipStream_t st)
{
    if (int rc = forward(bf16, master, w, batch, st))
        return rc;
    if (bf16)
        hipLaunchKernelGGL(k_loss<uint16_t>, dim3(blocks(batch, 256)), dim3(256), 0, st, w.out,
                           target, (int)batch, w.dout_f, (uint16_t *)w.dout_t, w.per_sample);
    else
        hipLaunchKernelGGL(k_loss<float>, dim3(blocks(batch, 256)), dim3(256), 0, st, w.out,
                           target, (int)batch, w.dout_f, (float *)w.dout_t, w.per_sample);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, w.per_sample, (int)batch,
                       1.0f / (float)batch, loss);
    return backward(bf16, master, w, batch, grad, st);
}

void adam_launch(float *master, float *m, float *v, const float *grad, int32_t step, float lr,
                 hipStream_t st)
{
    // 1 - beta and the bias corrections are formed in double: in float,
    // 1 - 0.999f is 1.3e-5 away from 0.001
    const double b1 = 0.9, b2 = 0.999;
    const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(kParams, 256)), dim3(256), 0, st, master, m, v, grad,
                       kParams, lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2),
                       1e-8f, (float)c1, (float)c2);
}

}  // namespace

extern "C" {

int mlp_grad(const float *master, const float *x, const float *target, int64_t batch,
             int32_t precision, float *grad, float *loss, void *workspace, size_t ws,
             void *stream)
{
    if (!master || !x || !target || !grad || !loss || !workspace)
        return fail(ME_EINVAL, "NULL argument");
    if (batch < 1 || ws < ws_bytes(batch))
        return fail(ME_ENOMEM, "workspace of %zu B too small for batch %lld", ws,
                    (long long)batch);
    Ws w = ws_layout(workspace, batch);
    hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(w.x, x, batch * kIn * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    return grad_pass(precision == 0, master, w, target, batch, grad, loss, st);
}

int mlp_adam(float *master, float *m, float *v, const float *grad, int32_t step, float lr,
             void *stream)
{
    if (!master || !m || !v || !grad || step < 1 || !(lr > 0))
        return fail(ME_EINVAL, "invalid Adam arguments");
    adam_launch(master, m, v, grad, step, lr, as_stream(stream));
    return check_launch("mlp_adam");
}

int mlp_draw_examples(uint64_t seed, int64_t first, int64_t n, const me_bounds *bounds,
                      float *params, float *target, void *stream)
{
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!params || !target)
        return fail(ME_EINVAL, "NULL array argument");
    hipLaunchKernelGGL(k_draw, dim3(blocks(n, 256)), dim3(256), 0, as_stream(stream), seed, first,
                       n, b, params, target);
    return check_launch("mlp_draw_examples");
}

int mlp_add_noise(uint64_t seed, int64_t first, const float *params, int64_t n,
                  const me_grid *grids, int32_t nlines, float sigma_rel, float *stokes,
                  void *stream)
{
    if (!grids || nlines < 1 || nlines > GENESIS_MAX_LINES)
        return fail(ME_EINVAL, "invalid grids");
    int L = 0;
    for (int i = 0; i < nlines; ++i)
        L += grids[i].n;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!params || !stokes)
        return fail(ME_EINVAL, "NULL array argument");
    hipLaunchKernelGGL(k_noise, dim3((unsigned)n), dim3(256), 0, as_stream(stream), seed, first,
                       params, n, L, sigma_rel, stokes);
    return check_launch("mlp_add_noise");
}

int mlp_unscale(const float *y, int64_t n, const me_bounds *bounds, float *params, void *stream)
{
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    if (n < 0)
        return fail(ME_EINVAL, "n must be >= 0");
    if (n == 0)
        return ME_OK;
    if (!y || !params)
        return fail(ME_EINVAL, "NULL array argument");
    hipLaunchKernelGGL(k_unscale, dim3(blocks(n * GENESIS_NPAR, 256)), dim3(256), 0,
                       as_stream(stream), y, n, b, params);
    return check_launch("mlp_unscale");
}

size_t mlp_train_workspace_bytes(int64_t batch)
{
    return batch > 0 ? train_ws_bytes(batch, kIn / 4) : 0;
}

int mlp_train(float *master, float *m, float *v, int32_t first_step, int32_t steps,
              int64_t batch, float lr, uint64_t seed, const me_line *lines, const me_grid *grids,
              int32_t nlines, const me_bounds *bounds, float sigma_rel, int32_t precision,
              float *losses, void *workspace, size_t ws, void *stream)
{
    if (!master || !m || !v || !losses || !workspace)
        return fail(ME_EINVAL, "NULL argument");
    if (first_step < 1 || steps < 0 || !(lr > 0) || !(sigma_rel >= 0))
        return fail(ME_EINVAL, "need first_step >= 1, steps >= 0, lr > 0, sigma_rel >= 0");
    if (!grids || nlines < 1 || nlines > GENESIS_MAX_LINES)
        return fail(ME_EINVAL, "invalid grids");
    int L = 0;
    for (int i = 0; i < nlines; ++i)
        L += grids[i].n;
    if (4 * L != kIn)
        return fail(ME_EINVAL, "the network takes 4 L = %d inputs, got L = %d", kIn, L);
    if (batch < 1 || batch > (1 << 20) || ws < train_ws_bytes(batch, L))
        return fail(ME_ENOMEM, "workspace of %zu B too small for batch %lld", ws,
                    (long long)batch);
    Bounds b;
    if (int rc = pack_bounds(bounds, b))
        return rc;
    hipStream_t st = as_stream(stream);
    const Ws w = ws_layout(workspace, batch);
    const TrainWs t = train_layout(workspace, batch, L);
    const bool bf16 = precision == 0;
    for (int32_t s = 0; s < steps; ++s) {
        const int32_t step = first_step + s;
        // examples (step - 1) * batch ... step * batch - 1 of the stream `seed`
        const int64_t first = (int64_t)(step - 1) * batch;
        hipLaunchKernelGGL(k_draw, dim3(blocks(batch, 256)), dim3(256), 0, st, seed, first, batch,
                           b, t.params, t.target);
        if (int rc = me_synth(t.params, batch, lines, grids, nlines, nullptr, t.stokes, stream))
            return rc;
        hipLaunchKernelGGL(k_noise, dim3((unsigned)batch), dim3(256), 0, st, seed, first,
                           t.params, batch, L, sigma_rel, t.stokes);
        hipLaunchKernelGGL(k_features, dim3((unsigned)batch), dim3(256), 0, st, t.stokes, batch,
                           L, w.x);
        if (int rc = grad_pass(bf16, master, w, t.target, batch, t.grad, losses + s, st))
            return rc;
        adam_launch(master, m, v, t.grad, step, lr, st);
    }
    return check_launch("mlp_train");
}

}  // extern "C"
