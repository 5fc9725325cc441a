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

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---- FP32 products (VALU; the reference-precision mode for gradient checks)

enum Epi : int { kFwdHidden = 0, kFwdOut = 1, kBwdHidden = 2, kGradW = 3 };

struct GemmArgs {
    const float *A, *B;
    int M, N, K;
    int lda, ldb;         // leading dimensions of A, B as stored
    const float *bias;    // [N]            (forward)
    const float *pre_in;  // [M][N]         (backward: pre-activation)
    float *outf;          // [M][N] pre-activation, output, error or gradient
    float *outt;          // [M][N] activation (kFwdHidden only)
};

// Epilogue of one accumulated element (m, n).
template <int EPI>
__device__ __forceinline__ void epilogue(const GemmArgs &a, int m, int n, float acc)
{
    if (m >= a.M || n >= a.N)
        return;
    const int64_t i = (int64_t)m * a.N + n;
    if (EPI == kFwdHidden) {
        const float pre = acc + a.bias[n];
        a.outf[i] = pre;
        a.outt[i] = gelu(pre);
    } else if (EPI == kFwdOut) {
        a.outf[i] = acc + a.bias[n];
    } else if (EPI == kBwdHidden) {
        a.outf[i] = acc * gelu_d(a.pre_in[i]);
    } else {
        a.outf[i] = acc;
    }
}

// FP32 reference-precision product on the VALU (gradient checks).
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs a)
{
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ float As[BK][BM + 1];
    __shared__ float Bs[BK][BN + 1];
    const float *A = a.A, *B = a.B;
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
            epilogue<EPI>(a, m0 + tm + i, n0 + tn + j, acc[i][j]);
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

// Loss: mean over the batch of sum_j d_j^2 with d = out - target, the azimuth
// (j = 2) taken modulo 1 (its 180-degree period).  Writes dL/dout and the
// per-sample loss.
__global__ void k_loss(const float *out, const float *target, int B, float *dout,
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
        dout[b * kOut + j] = 2.0f * d / (float)B;
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

// ---- BF16 products on the matrix cores ------------------------------------
//
// Every product is C[M][N] = A[M][K] B[K][N], staged in LDS as [rows][k]
// (k contiguous, a pitch of 72 elements), so that an MFMA operand is one
// 16-byte LDS read: A's rows are the M index, B's rows the N index.  An
// operand stored with k contiguous in memory (KC) is copied in 16-byte
// chunks; one stored with its rows contiguous ([K][rows]) is transposed on
// the way into LDS.  Workgroup: 256 threads, 4 waves in 2 x 2, output tile
// 64 x 64, wave tile 32 x 32 (one v_mfma_f32_32x32x16_bf16 accumulator);
// k step 64 through two LDS buffers, with the operands of the next kStages
// steps in flight in registers.  The tile is small so that the products of a
// training batch (4096 x 512 outputs) give two workgroups per compute unit,
// whose waves hide each other's memory latency.
//
// The loaders read whole 16-byte chunks only.  For a KC operand the chunk
// runs along k (K a multiple of 8); for a row-contiguous one it runs along the
// rows (their count a multiple of 8).  A chunk outside the operand reads the
// operand's first chunk and is zeroed when stored, so every path issues the
// same loads and each store waits only for its own step's loads.
constexpr int kBM = 64, kBN = 64, kBK = 64, kPitch = kBK + 8;
constexpr int kAcc = kBM / 64;  // 32-row accumulators per wave
// register stages of operands in flight (even: stage p fills LDS buffer p % 2)
constexpr int kStages = 2;
// most k ranges a weight-gradient product is split into
constexpr int kSplitMax = 8;
// the output layer's 9 rows padded to 16 (a multiple of the loaders' chunk)
constexpr int kOutPad = 16;

__device__ __forceinline__ bf16x8 keep(bf16x8 v, bool whole)
{
    const bf16x8 z = {0};
    return whole ? v : z;
}

template <bool KC, int ROWS>
struct Stage;

// k contiguous ([rows][ld]): thread t owns chunks q = t + 256 j, row q / 8,
// k 8 (q % 8) .. + 7; 8 lanes fill one 128-byte LDS row segment
template <int ROWS>
struct Stage<true, ROWS> {
    static constexpr int kN = ROWS / 32;
    bf16x8 v[kN];
    bool ok[kN];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ X, int ld, int rows, int ke,
                                         int row0, int k0, int tid)
    {
#pragma unroll
        for (int j = 0; j < kN; ++j) {
            const int q = tid + 256 * j;
            const int gr = row0 + (q >> 3), gc = k0 + (q & 7) * 8;
            ok[j] = gr < rows && gc < ke;
            v[j] = *(const bf16x8 *)(X + (ok[j] ? (int64_t)gr * ld + gc : 0));
        }
    }

    __device__ __forceinline__ void store(uint16_t (*T)[kPitch], int tid) const
    {
#pragma unroll
        for (int j = 0; j < kN; ++j) {
            const int q = tid + 256 * j;
            *(bf16x8 *)&T[q >> 3][(q & 7) * 8] = keep(v[j], ok[j]);
        }
    }
};

// rows contiguous ([K][ld]): per 64-row group g, thread t loads rows
// 64 g + 8 (t / 32) .. + 7 of the k columns 2 (t % 32) and 2 (t % 32) + 1,
// pairs the two k of each row into one dword and writes 8 dwords; the 32
// lanes of a half-wave write 128 consecutive bytes of one LDS row
template <int ROWS>
struct Stage<false, ROWS> {
    static constexpr int kG = ROWS / 64;
    bf16x8 v[kG][2];
    bool ok[kG][2];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ X, int ld, int rows, int ke,
                                         int row0, int k0, int tid)
    {
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int gr = row0 + 64 * g + 8 * (tid >> 5);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int gc = k0 + 2 * (tid & 31) + j;
                ok[g][j] = gc < ke && gr < rows;
                v[g][j] = *(const bf16x8 *)(X + (ok[g][j] ? (int64_t)gc * ld + gr : 0));
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t (*T)[kPitch], int tid) const
    {
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const int r = 64 * g + 8 * (tid >> 5), c = 2 * (tid & 31);
            const bf16x8 v0 = keep(v[g][0], ok[g][0]);
            const bf16x8 v1 = keep(v[g][1], ok[g][1]);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *(uint32_t *)&T[r + e][c] =
                    (uint32_t)(uint16_t)v0[e] | ((uint32_t)(uint16_t)v1[e] << 16);
        }
    }
};

// The products of a training step (layer l maps kDims[l] inputs to
// kDims[l + 1] outputs; X its input, d its output error; Wp the output
// layer's weights as 16 rows, rows 9-15 zero):
//   kJobFwd   pre = X W^T + b, act = gelu(pre)      A = X [B][in] (KC), B = W [out][in] (KC)
//   kJobOut   y = act Wp^T + b, with the loss and g = dL/dy in the epilogue
//                                                 A = act [B][512] (KC), B = Wp [16][512] (KC)
//   kJobBwd   e = (d W) * gelu'(pre of the layer below)
//                                                 A = d [B][out] (KC), B = W [out][in] (rows)
//   kJobGradW dW = d^T X, split over k = batch    A = d [B][out] (rows), B = X [B][in] (rows)
enum Job : int { kJobFwd = 0, kJobBwd = 1, kJobGradW = 2, kJobOut = 3 };

template <int J>
struct JobKind {
    static constexpr bool kca = J != kJobGradW, kcb = J == kJobFwd || J == kJobOut;
};

struct MmJob {
    const uint16_t *A, *B;
    int M, N, K, lda, ldb;
    int tiles_m, tiles_n, kper;  // kper: k range of one split (kJobGradW), a multiple of kBK
    int nblocks;                 // tiles_m tiles_n splits
    const float *bias;           // kJobFwd: [N]; kJobOut: [9]
    float *pre;                  // kJobFwd: [M][N] pre-activation, or NULL
    uint16_t *out;               // kJobFwd: gelu(pre); kJobBwd: e; [M][N] bf16
    const float *pre_in;         // kJobBwd: [M][N]
    float *colsum;               // kJobBwd: [tiles_m][N], sum of e over each tile's rows
    float *part;                 // kJobGradW: [splits][M][N]
    // kJobOut: y [M][9]; with a target [M][9] (training) also g16 = bf16(g)
    // [M][16] (zero after column 9) and per tile the sums of g [tiles_m][9]
    // and of the per-sample loss [tiles_m]
    float *y;
    const float *target;
    uint16_t *g16;
    float *gsum, *lsum;
};

struct MmArgs {
    MmJob j[2];
};

template <bool KCA, bool KCB>
__device__ __forceinline__ void mm_step(Stage<KCA, kBM> &sa, Stage<KCB, kBN> &sb,
                                        uint16_t (*As)[kPitch], uint16_t (*Bs)[kPitch],
                                        const MmJob &j, int ke, int m0, int n0, int knext, int tid,
                                        int lane, int wm, int wn, f32x16 (&acc)[kAcc])
{
    sa.store(As, tid);
    sb.store(Bs, tid);
    __syncthreads();
    sa.load(j.A, j.lda, j.M, ke, m0, knext, tid);
    sb.load(j.B, j.ldb, j.N, ke, n0, knext, tid);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 16) {
        const int kr = kk + 8 * (lane >> 5);
        const bf16x8 bv = *(const bf16x8 *)&Bs[wn + (lane & 31)][kr];
#pragma unroll
        for (int i = 0; i < kAcc; ++i) {
            const bf16x8 av = *(const bf16x8 *)&As[wm + 32 * i + (lane & 31)][kr];
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[i], 0, 0, 0);
        }
    }
}

struct MmShared {
    uint16_t A[2][kBM][kPitch];
    uint16_t B[2][kBN][kPitch];
    float col[2][kBN];
};

// accumulator element r of lane l: row 8 (r / 4) + 4 (l / 32) + r % 4,
// column l % 32 of the 32 x 32 tile
__device__ __forceinline__ int acc_row(int i, int r, int lane)
{
    return 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// kJobOut epilogue: the tile's 16 output columns go through LDS, then one
// thread per sample forms y, the loss terms and g; the tile's sums of g and
// of the loss are added in row order.
__device__ __forceinline__ void out_epilogue(const MmJob &j, const f32x16 (&acc)[kAcc], int tm,
                                             int m0, int wm, int wn, int tid, int lane,
                                             MmShared &sh)
{
    __syncthreads();  // the last step's operands may still be read
    float(*Y)[kOutPad + 1] = (float(*)[kOutPad + 1]) & sh.A[0][0][0];
    float *G = (float *)&sh.B[0][0][0];  // [kBM][9] g, then [kBM] loss
    if (wn == 0 && (lane & 31) < kOutPad) {
#pragma unroll
        for (int i = 0; i < kAcc; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                Y[wm + acc_row(i, r, lane)][lane & 31] = acc[i][r];
    }
    __syncthreads();
    const bool train = j.target != nullptr;
    if (tid < kBM) {
        const int m = m0 + tid;
        const int64_t mc = min(m, j.M - 1);
        float tv[kOut];
        if (train) {
#pragma unroll
            for (int c = 0; c < kOut; ++c)
                tv[c] = j.target[mc * kOut + c];
        }
        float s = 0.0f;
        uint32_t gq[kOutPad / 2] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < kOut; ++c) {
            const float yv = Y[tid][c] + j.bias[c];
            float gc = 0.0f;
            if (m < j.M) {
                j.y[(int64_t)m * kOut + c] = yv;
                if (train) {
                    float d = yv - tv[c];
                    if (c == 2)
                        d = d - rintf(d);
                    s = fmaf(d, d, s);
                    gc = 2.0f * d / (float)j.M;
                }
            }
            gq[c >> 1] |= (uint32_t)f2bf(gc) << (16 * (c & 1));
            G[tid * kOut + c] = gc;
        }
        G[kBM * kOut + tid] = s;
        if (train && m < j.M) {
            uint4 *dst = (uint4 *)(j.g16 + (int64_t)m * kOutPad);
            dst[0] = make_uint4(gq[0], gq[1], gq[2], gq[3]);
            dst[1] = make_uint4(gq[4], gq[5], gq[6], gq[7]);
        }
    }
    if (!train)
        return;
    __syncthreads();
    if (tid < kOut) {
        float s = 0.0f;
        for (int r = 0; r < kBM; ++r)
            s += G[r * kOut + tid];
        j.gsum[(int64_t)tm * kOut + tid] = s;
    } else if (tid == kOut) {
        float s = 0.0f;
        for (int r = 0; r < kBM; ++r)
            s += G[kBM * kOut + r];
        j.lsum[tm] = s;
    }
}

template <int J>
__device__ __forceinline__ void mm_run(const MmJob &j, int local, MmShared &sh)
{
    constexpr bool KCA = JobKind<J>::kca, KCB = JobKind<J>::kcb;
    // workgroups are dealt to the 8 XCDs in turn: give each XCD a contiguous
    // range of tiles (n fastest, then m, then split) so that the tiles
    // sharing an A block, or a k range, share that XCD's L2
    int t = local;
    if (j.nblocks % 8 == 0)
        t = (local & 7) * (j.nblocks >> 3) + (local >> 3);
    const int tn = t % j.tiles_n, tm = (t / j.tiles_n) % j.tiles_m;
    const int z = t / (j.tiles_n * j.tiles_m);
    const int m0 = tm * kBM, n0 = tn * kBN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * (kBM / 2), wn = (wave & 1) * 32;
    const int kb = J == kJobGradW ? z * j.kper : 0;
    const int ke = J == kJobGradW ? min(j.K, kb + j.kper) : j.K;
    Stage<KCA, kBM> sa[kStages];
    Stage<KCB, kBN> sb[kStages];
#pragma unroll
    for (int p = 0; p < kStages; ++p) {
        sa[p].load(j.A, j.lda, j.M, ke, m0, kb + p * kBK, tid);
        sb[p].load(j.B, j.ldb, j.N, ke, n0, kb + p * kBK, tid);
    }
    f32x16 acc[kAcc];
#pragma unroll
    for (int i = 0; i < kAcc; ++i)
        acc[i] = f32x16{0};
    const int nsteps = ke > kb ? (ke - kb + kBK - 1) / kBK : 0;
    for (int s = 0; s < nsteps; s += kStages) {
#pragma unroll
        for (int p = 0; p < kStages; ++p)
            if (s + p < nsteps)
                mm_step(sa[p], sb[p], sh.A[p & 1], sh.B[p & 1], j, ke, m0, n0,
                        kb + (s + p + kStages) * kBK, tid, lane, wm, wn, acc);
    }
    if (J == kJobOut) {
        out_epilogue(j, acc, tm, m0, wm, wn, tid, lane, sh);
        return;
    }

    const int n = n0 + wn + (lane & 31);
    // the backward epilogue's pre-activations, all loads issued before any
    // is used (rows past the end read the last row and are not used)
    float pin[kAcc][16];
    if (J == kJobBwd) {
#pragma unroll
        for (int i = 0; i < kAcc; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                pin[i][r] = j.pre_in[(int64_t)min(m0 + wm + acc_row(i, r, lane), j.M - 1) * j.N + n];
    }
    float cs = 0.0f;
#pragma unroll
    for (int i = 0; i < kAcc; ++i) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = m0 + wm + acc_row(i, r, lane);
            const int64_t e = (int64_t)m * j.N + n;
            if (J == kJobFwd) {
                if (m < j.M) {
                    const float pre = acc[i][r] + j.bias[n];
                    if (j.pre)
                        j.pre[e] = pre;
                    j.out[e] = f2bf(gelu(pre));
                }
            } else if (J == kJobBwd) {
                if (m < j.M) {
                    const float d = acc[i][r] * gelu_d(pin[i][r]);
                    j.out[e] = f2bf(d);
                    cs += d;
                }
            } else {
                if (m < j.M)
                    j.part[(int64_t)z * j.M * j.N + e] = acc[i][r];
            }
        }
    }
    if (J == kJobBwd) {
        // column sums over the tile's rows in a fixed order: each lane's
        // rows, then the two half-waves, then the two waves of a column
        cs += __shfl_xor(cs, 32);
        if (lane < 32)
            sh.col[wave >> 1][wn + lane] = cs;
        __syncthreads();
        if (tid < kBN)
            j.colsum[(int64_t)tm * j.N + n0 + tid] = sh.col[0][tid] + sh.col[1][tid];
    }
}

// One launch runs the workgroups of up to two independent products: blocks
// [0, j[0].nblocks) the first, the rest the second.
template <int J0, int J1>
__global__ __launch_bounds__(256) void k_mm(MmArgs a)
{
    __shared__ __align__(16) MmShared sh;
    const int b = blockIdx.x;
    if (b < a.j[0].nblocks)
        mm_run<J0>(a.j[0], b, sh);
    else
        mm_run<J1>(a.j[1], b - a.j[0].nblocks, sh);
}

// BF16 operands of a pass, 4 values per thread: blocks [0, wblocks) round
// the master weights (n_w values), the next pblocks write the output
// layer's weights as 16 rows (rows 9-15 zero), the rest round the input
// (n_x values, a multiple of 4).
__global__ __launch_bounds__(256) void k_prep(const float *__restrict__ w, int64_t n_w,
                                              uint16_t *__restrict__ wb, int wblocks,
                                              uint16_t *__restrict__ wpad, int pblocks,
                                              const float *__restrict__ x, int64_t n_x,
                                              uint16_t *__restrict__ xb)
{
    const int blk = blockIdx.x;
    if (blk >= wblocks && blk < wblocks + pblocks) {
        const int i = 4 * ((blk - wblocks) * 256 + (int)threadIdx.x);
        const float *w3 = w + w_off(kLayers - 1);
        for (int e = i; e < min(i + 4, kOutPad * kHid); ++e)
            wpad[e] = e < kOut * kHid ? f2bf(w3[e]) : (uint16_t)0;
        return;
    }
    const bool is_w = blk < wblocks;
    const int64_t i = 4 * ((int64_t)(is_w ? blk : blk - wblocks - pblocks) * 256 + threadIdx.x);
    const float *in = is_w ? w : x;
    uint16_t *out = is_w ? wb : xb;
    const int64_t n = is_w ? n_w : n_x;
    if (i + 4 <= n && ((uintptr_t)in & 15) == 0 && ((uintptr_t)out & 7) == 0) {
        const float4 v = *(const float4 *)(in + i);
        uint2 o;
        o.x = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
        o.y = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
        *(uint2 *)(out + i) = o;
    } else {
        for (int64_t e = i; e < min(i + 4, n); ++e)
            out[e] = f2bf(in[e]);
    }
}

// The gradient from the partials, each element summed in a fixed order.
// Blocks [0, nsum): sums of many terms (the biases and the loss): a block
// takes 64 outputs of one sum, its four waves the terms q = w, w + 4, ...,
// then the four wave sums are added in order.  The rest: the weights, four
// consecutive elements a thread, summed over the k splits.
struct SumSeg {
    const float *src;  // term q of output o at src[q * stride + o]
    int nout, nterms, stride;
    float scale;
    float *dst;
};

struct ReduceArgs {
    SumSeg seg[5];
    int seg_block[6];     // first block of each sum segment; seg_block[5] = nsum
    const float *part[4]; // [splits][rows][in]: layers 0-2, then the output layer (16 rows)
    int splits[4];
    int wblock[5];        // first block of each layer's weights (after nsum); wblock[4] = grid
    float *grad;
};

__global__ __launch_bounds__(256) void k_grad_reduce(ReduceArgs a)
{
    __shared__ float red[4][64];
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b < a.seg_block[5]) {
        int k = 0;
        while (b >= a.seg_block[k + 1])
            ++k;
        const SumSeg &sg = a.seg[k];
        const int w = tid >> 6, o = (b - a.seg_block[k]) * 64 + (tid & 63);
        float s = 0.0f;
        if (o < sg.nout) {
            for (int q0 = w; q0 < sg.nterms; q0 += 32) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + 4 * u;
                    v[u] = q < sg.nterms ? sg.src[(int64_t)q * sg.stride + o] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    s += v[u];
            }
        }
        red[w][tid & 63] = s;
        __syncthreads();
        if (w == 0 && o < sg.nout)
            sg.dst[o] = (((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid]) * sg.scale;
        return;
    }
    int l = 0;
    while (b >= a.wblock[l + 1])
        ++l;
    const int64_t n = (int64_t)kDims[l + 1] * kDims[l];
    const int64_t i = 4 * ((int64_t)(b - a.wblock[l]) * 256 + tid);
    if (i >= n)
        return;
    // the output layer's partials hold 16 rows of which the first 9 are its
    const int64_t pstride = l < kLayers - 1 ? n : (int64_t)kOutPad * kDims[l];
    const float4 *p = (const float4 *)(a.part[l] + i);
    float4 t[kSplitMax];
#pragma unroll
    for (int z = 0; z < kSplitMax; ++z)
        t[z] = z < a.splits[l] ? p[z * pstride / 4] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 s = t[0];
#pragma unroll
    for (int z = 1; z < kSplitMax; ++z) {
        if (z < a.splits[l]) {
            s.x += t[z].x;
            s.y += t[z].y;
            s.z += t[z].z;
            s.w += t[z].w;
        }
    }
    float *g = a.grad + w_off(l) + i;
    if (((uintptr_t)a.grad & 15) == 0) {
        *(float4 *)g = s;
    } else {
        g[0] = s.x;
        g[1] = s.y;
        g[2] = s.z;
        g[3] = s.w;
    }
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

// Split-K factor of a weight-gradient product with `tiles` output tiles and
// K = batch: about 512 workgroups, at least one k step per split.
int split_of(int tiles, int64_t K)
{
    int s = (512 + tiles - 1) / tiles;
    s = (int)std::min<int64_t>(s, (K + kBK - 1) / kBK);
    return std::max(1, std::min(s, kSplitMax));
}

int row_tiles(int64_t B) { return (int)((B + kBM - 1) / kBM); }

struct Ws {
    // the forward pass (also the layout of the no-allocation forward's scratch)
    uint16_t *wbf;       // bf16 weights [kParams]
    uint16_t *wpad;      // bf16 output-layer weights as 16 rows [16][512], rows 9-15 zero
    float *x;            // input [B][1024] f32 (the training examples' features)
    uint16_t *xb;        // input bf16
    float *pre[3];       // pre-activations [B][512]
    void *act[3];        // activations [B][512] (f32, or bf16 on the matrix cores)
    float *out;          // [B][9]
    // the backward pass
    float *dout;         // [B][9] dL/dy (FP32 mode)
    void *dh[2];         // [B][512] errors of two consecutive layers (f32 or bf16)
    float *per_sample;   // [B] (FP32 mode)
    uint16_t *g16;       // dL/dy in bf16, 16 columns [B][16]
    float *gsum, *lsum;  // per row tile: sums of dL/dy [tiles][9] and of the loss [tiles]
    float *part[4];      // split-K weight-gradient partials [kSplitMax][out][in] of layers
                         // 0-2 and [kSplitMax][16][512] of the output layer
    float *colsum[3];    // bias-gradient partials of layers 0-2 [row tiles][512]
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// every buffer above, in this order (the forward's first)
template <typename F>
void ws_walk(int64_t B, bool forward_only, F &&take)
{
    const size_t tiles = row_tiles(B);
    take(kParams * 2);
    take(kOutPad * kHid * 2);
    take(B * kIn * 4);
    take(B * kIn * 2);
    for (int i = 0; i < 3; ++i) {
        take(B * kHid * 4);
        take(B * kHid * 4);
    }
    take(B * kOut * 4);
    if (forward_only)
        return;
    take(B * kOut * 4);
    take(B * kHid * 4);
    take(B * kHid * 4);
    take(B * 4);
    take(B * kOutPad * 2);
    take(tiles * kOut * 4);
    take(tiles * 4);
    for (int l = 0; l < 3; ++l)
        take((size_t)kSplitMax * kDims[l + 1] * kDims[l] * 4);
    take((size_t)kSplitMax * kOutPad * kHid * 4);
    for (int l = 0; l < 3; ++l)
        take(tiles * kHid * 4);
}

size_t ws_bytes(int64_t B)
{
    size_t s = 0;
    ws_walk(B, false, [&](size_t n) { s += al(n); });
    return s;
}

// The forward pass alone needs the BF16 weights, the input (FP32 and BF16),
// the three hidden layers (pre-activation and activation) and the output,
// placed as ws_layout places them.
size_t fwd_bytes(int64_t B)
{
    size_t s = 0;
    ws_walk(B, true, [&](size_t n) { s += al(n); });
    return s;
}

Ws layout(void *base, int64_t B, bool forward_only)
{
    std::vector<void *> p;
    char *c = (char *)base;
    ws_walk(B, forward_only, [&](size_t n) {
        p.push_back(c);
        c += al(n);
    });
    Ws w{};
    int i = 0;
    w.wbf = (uint16_t *)p[i++];
    w.wpad = (uint16_t *)p[i++];
    w.x = (float *)p[i++];
    w.xb = (uint16_t *)p[i++];
    for (int l = 0; l < 3; ++l) {
        w.pre[l] = (float *)p[i++];
        w.act[l] = p[i++];
    }
    w.out = (float *)p[i++];
    if (forward_only)
        return w;
    w.dout = (float *)p[i++];
    w.dh[0] = p[i++];
    w.dh[1] = p[i++];
    w.per_sample = (float *)p[i++];
    w.g16 = (uint16_t *)p[i++];
    w.gsum = (float *)p[i++];
    w.lsum = (float *)p[i++];
    for (int l = 0; l < 4; ++l)
        w.part[l] = (float *)p[i++];
    for (int l = 0; l < 3; ++l)
        w.colsum[l] = (float *)p[i++];
    return w;
}

Ws ws_layout(void *base, int64_t B) { return layout(base, B, false); }
Ws fwd_layout(void *base, int64_t B) { return layout(base, B, true); }

// Scratch of mlp_forward_noalloc: one forward workspace of kNoAllocRows rows
// per device, a file-scope device array.  Host code must not pass the array's
// name to a kernel (that is a host-side stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoAllocRows = 1024;
constexpr size_t kNoAllocBytes = (kParams * 2 + 255) / 256 * 256 + kOutPad * kHid * 2 +
                                 kNoAllocRows * kIn * 4 + kNoAllocRows * kIn * 2 +
                                 6 * kNoAllocRows * kHid * 4 +
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

// ---- passes ---------------------------------------------------------------

int blocks(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

template <int EPI, bool TA, bool TB>
int gemm_f32(const GemmArgs &a, hipStream_t st)
{
    const dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
    hipLaunchKernelGGL((k_gemm_f32<TA, TB, EPI>), grid, dim3(256), 0, st, a);
    return check_launch("mlp gemm");
}

// FP32 forward from x [B][1024]
int forward_f32(const float *master, const float *x, const Ws &w, int64_t B, hipStream_t st)
{
    const float *in = x;
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs a{};
        a.A = in;
        a.B = master + w_off(l);
        a.M = (int)B;
        a.N = kDims[l + 1];
        a.K = kDims[l];
        a.lda = kDims[l];
        a.ldb = kDims[l];  // W stored [out][in] = B transposed
        a.bias = master + b_off(l);
        int rc;
        if (l < kLayers - 1) {
            a.outf = w.pre[l];
            a.outt = (float *)w.act[l];
            rc = gemm_f32<kFwdHidden, false, true>(a, st);
            in = (const float *)w.act[l];
        } else {
            a.outf = w.out;
            rc = gemm_f32<kFwdOut, false, true>(a, st);
        }
        if (rc)
            return rc;
    }
    return ME_OK;
}

// FP32 backward from dL/dy in w.dout
int backward_f32(const float *master, const float *x, const Ws &w, int64_t B, float *grad,
                 hipStream_t st)
{
    const float *d = w.dout;
    int buf = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int nout = kDims[l + 1], nin = kDims[l];
        GemmArgs g{};
        g.A = d;  // d [B][nout] used transposed: A[m = out][k = b]
        g.B = l == 0 ? x : (const float *)w.act[l - 1];  // X [B][nin]: B[k = b][n = in]
        g.M = nout;
        g.N = nin;
        g.K = (int)B;
        g.lda = nout;
        g.ldb = nin;
        g.outf = grad + w_off(l);
        if (int rc = gemm_f32<kGradW, true, false>(g, st))
            return rc;
        hipLaunchKernelGGL(k_colsum, dim3(blocks(nout, 64)), dim3(1024), 0, st, d, (int)B, nout,
                           grad + b_off(l));
        if (l == 0)
            break;
        GemmArgs e{};
        e.A = d;  // d [B][nout]
        e.B = master + w_off(l);
        e.M = (int)B;
        e.N = nin;
        e.K = nout;
        e.lda = nout;
        e.ldb = nin;  // W [out][in] = B[k = out][n = in] row-major
        e.pre_in = w.pre[l - 1];
        e.outf = (float *)w.dh[buf];
        if (int rc = gemm_f32<kBwdHidden, false, false>(e, st))
            return rc;
        d = (const float *)w.dh[buf];
        buf ^= 1;
    }
    return check_launch("mlp backward");
}

static_assert(kHid % kBM == 0 && kHid % kBN == 0 && kIn % kBN == 0 && kIn % 8 == 0,
              "the layer widths must fill whole tiles");

MmJob fwd_job(const uint16_t *X, const uint16_t *W, int64_t B, int l, const float *bias,
              float *pre, uint16_t *out)
{
    MmJob j{};
    j.A = X;
    j.B = W;
    j.M = (int)B;
    j.N = kDims[l + 1];
    j.K = kDims[l];
    j.lda = j.K;
    j.ldb = j.K;
    j.tiles_m = row_tiles(B);
    j.tiles_n = j.N / kBN;
    j.nblocks = j.tiles_m * j.tiles_n;
    j.bias = bias;
    j.pre = pre;
    j.out = out;
    return j;
}

// e = (d W_l) * gelu'(pre_{l-1}): M = B, N = inputs of layer l, K = its
// outputs (kOutPad for the output layer, whose W and d carry 16 rows)
MmJob bwd_job(const uint16_t *d, const uint16_t *W, int64_t B, int l, const float *pre_in,
              uint16_t *out, float *colsum)
{
    MmJob j{};
    j.A = d;
    j.B = W;
    j.M = (int)B;
    j.N = kDims[l];
    j.K = l < kLayers - 1 ? kDims[l + 1] : kOutPad;
    j.lda = j.K;
    j.ldb = j.N;
    j.tiles_m = row_tiles(B);
    j.tiles_n = j.N / kBN;
    j.nblocks = j.tiles_m * j.tiles_n;
    j.pre_in = pre_in;
    j.out = out;
    j.colsum = colsum;
    return j;
}

// dW_l = d^T X: M = outputs of layer l (rows of d, kOutPad for the output
// layer), N = its inputs, K = B split in ranges
MmJob gradw_job(const uint16_t *d, const uint16_t *X, int64_t B, int l, float *part,
                int *splits)
{
    MmJob j{};
    j.A = d;
    j.B = X;
    j.M = l < kLayers - 1 ? kDims[l + 1] : kOutPad;
    j.N = kDims[l];
    j.K = (int)B;
    j.lda = j.M;
    j.ldb = j.N;
    j.tiles_m = (j.M + kBM - 1) / kBM;
    j.tiles_n = j.N / kBN;
    const int tiles = j.tiles_m * j.tiles_n;
    const int s = split_of(tiles, B);
    j.kper = (int)((((B + s - 1) / s) + kBK - 1) / kBK * kBK);
    *splits = (int)((B + j.kper - 1) / j.kper);
    j.nblocks = tiles * *splits;
    j.part = part;
    return j;
}

template <int J0, int J1>
int launch_mm(const MmJob &a, const MmJob &b, hipStream_t st, const char *what)
{
    const MmArgs args{{a, b}};
    hipLaunchKernelGGL((k_mm<J0, J1>), dim3(a.nblocks + b.nblocks), dim3(256), 0, st, args);
    return check_launch(what);
}

// y = act W^T + b for the output layer (W as 16 rows), with the loss terms
// when a target is given
MmJob out_job(const Ws &w, const float *master, int64_t B, float *y, const float *target)
{
    MmJob j{};
    j.A = (const uint16_t *)w.act[kLayers - 2];
    j.B = w.wpad;
    j.M = (int)B;
    j.N = kOutPad;
    j.K = kHid;
    j.lda = kHid;
    j.ldb = kHid;
    j.tiles_m = row_tiles(B);
    j.tiles_n = 1;
    j.nblocks = j.tiles_m;
    j.bias = master + b_off(kLayers - 1);
    j.y = y;
    j.target = target;
    j.g16 = w.g16;
    j.gsum = w.gsum;
    j.lsum = w.lsum;
    return j;
}

// BF16 forward: operands rounded to bfloat16, the three hidden layers on the
// matrix cores (pre-activations kept for a backward pass), then the output
// layer (with the loss terms when a target is given) into y
int forward_bf16(const float *master, const float *x, const Ws &w, int64_t B, bool keep_pre,
                 float *y, const float *target, hipStream_t st)
{
    const int wblocks = blocks((kParams + 3) / 4, 256);
    const int pblocks = blocks(kOutPad * kHid / 4, 256);
    hipLaunchKernelGGL(k_prep, dim3(wblocks + pblocks + blocks(B * kIn / 4, 256)), dim3(256), 0,
                       st, master, kParams, w.wbf, wblocks, w.wpad, pblocks, x, B * kIn, w.xb);
    if (int rc = check_launch("mlp operands"))
        return rc;
    const uint16_t *in = w.xb;
    for (int l = 0; l < kLayers - 1; ++l) {
        const MmJob j = fwd_job(in, w.wbf + w_off(l), B, l, master + b_off(l),
                                keep_pre ? w.pre[l] : nullptr, (uint16_t *)w.act[l]);
        if (int rc = launch_mm<kJobFwd, kJobFwd>(j, MmJob{}, st, "mlp forward product"))
            return rc;
        in = (const uint16_t *)w.act[l];
    }
    return launch_mm<kJobOut, kJobOut>(out_job(w, master, B, y, target), MmJob{}, st,
                                       "mlp output layer");
}

// BF16 loss and gradient: forward with the output layer's loss terms, then
// the backward products two to a launch (a weight gradient with the next
// error), the input layer's weight gradient, and the reduction of every
// partial into the gradient.
int grad_bf16(const float *master, const float *x, const Ws &w, const float *target, int64_t B,
              float *grad, float *loss, hipStream_t st)
{
    if (int rc = forward_bf16(master, x, w, B, true, w.out, target, st))
        return rc;
    uint16_t *e0 = (uint16_t *)w.dh[0], *e1 = (uint16_t *)w.dh[1];
    const uint16_t *act0 = (const uint16_t *)w.act[0], *act1 = (const uint16_t *)w.act[1];
    const uint16_t *act2 = (const uint16_t *)w.act[2];
    int S[4];
    const MmJob g3 = gradw_job(w.g16, act2, B, 3, w.part[3], &S[3]);
    const MmJob b3 = bwd_job(w.g16, w.wpad, B, 3, w.pre[2], e0, w.colsum[2]);
    if (int rc = launch_mm<kJobGradW, kJobBwd>(g3, b3, st, "mlp backward (layer 3)"))
        return rc;
    const MmJob g2 = gradw_job(e0, act1, B, 2, w.part[2], &S[2]);
    const MmJob b2 = bwd_job(e0, w.wbf + w_off(2), B, 2, w.pre[1], e1, w.colsum[1]);
    if (int rc = launch_mm<kJobGradW, kJobBwd>(g2, b2, st, "mlp backward (layer 2)"))
        return rc;
    const MmJob g1 = gradw_job(e1, act0, B, 1, w.part[1], &S[1]);
    const MmJob b1 = bwd_job(e1, w.wbf + w_off(1), B, 1, w.pre[0], e0, w.colsum[0]);
    if (int rc = launch_mm<kJobGradW, kJobBwd>(g1, b1, st, "mlp backward (layer 1)"))
        return rc;
    const MmJob g0 = gradw_job(e0, w.xb, B, 0, w.part[0], &S[0]);
    if (int rc = launch_mm<kJobGradW, kJobGradW>(g0, MmJob{}, st, "mlp backward (layer 0)"))
        return rc;
    ReduceArgs r{};
    const int tiles = row_tiles(B);
    for (int l = 0; l < 3; ++l)
        r.seg[l] = SumSeg{w.colsum[l], kHid, tiles, kHid, 1.0f, grad + b_off(l)};
    r.seg[3] = SumSeg{w.gsum, kOut, tiles, kOut, 1.0f, grad + b_off(3)};
    r.seg[4] = SumSeg{w.lsum, 1, tiles, 1, 1.0f / (float)B, loss};
    r.seg_block[0] = 0;
    for (int k = 0; k < 5; ++k)
        r.seg_block[k + 1] = r.seg_block[k] + (r.seg[k].nout + 63) / 64;
    r.wblock[0] = r.seg_block[5];
    for (int l = 0; l < kLayers; ++l) {
        r.part[l] = w.part[l];
        r.splits[l] = S[l];
        r.wblock[l + 1] = r.wblock[l] + blocks((int64_t)kDims[l + 1] * kDims[l], 1024);
    }
    r.grad = grad;
    hipLaunchKernelGGL(k_grad_reduce, dim3(r.wblock[kLayers]), dim3(256), 0, st, r);
    return check_launch("mlp gradient reduction");
}

// forward of n rows into y: BF16 on the matrix cores (precision 0) or FP32
int forward_into(const float *master, const float *x, int64_t n, bool bf16, const Ws &w,
                 float *y, hipStream_t st)
{
    if (bf16)
        return forward_bf16(master, x, w, n, false, y, nullptr, st);
    if (int rc = forward_f32(master, x, w, n, st))
        return rc;
    if (hipMemcpyAsync(y, w.out, n * kOut * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(ME_EHIP, "copy failed");
    return ME_OK;
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
    return forward_into(master, x, n, precision == 0, ws_layout(workspace, n), y,
                        as_stream(stream));
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
    return forward_into(master, x, n, precision == 0, fwd_layout(base, n), y, as_stream(stream));
}

}  // extern "C"

namespace {

// loss and gradient of one batch with features x [B][1024]
int grad_pass(bool bf16, const float *master, const float *x, const Ws &w, const float *target,
              int64_t batch, float *grad, float *loss, hipStream_t st)
{
    if (bf16)
        return grad_bf16(master, x, w, target, batch, grad, loss, st);
    if (int rc = forward_f32(master, x, w, batch, st))
        return rc;
    hipLaunchKernelGGL(k_loss, dim3(blocks(batch, 256)), dim3(256), 0, st, w.out, target,
                       (int)batch, w.dout, w.per_sample);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, w.per_sample, (int)batch,
                       1.0f / (float)batch, loss);
    return backward_f32(master, x, w, batch, grad, st);
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
    return grad_pass(precision == 0, master, x, ws_layout(workspace, batch), target, batch, grad,
                     loss, as_stream(stream));
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
        if (int rc = grad_pass(bf16, master, w.x, w, t.target, batch, t.grad, losses + s, st))
            return rc;
        adam_launch(master, m, v, t.grad, step, lr, st);
    }
    return check_launch("mlp_train");
}

}  // extern "C"
