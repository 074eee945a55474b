// Warm-start network for parametric LPs: forward, backward and Adam on the
// GPU with hand-written kernels.
//
// The network maps a sketch of an instance's perturbation (in_dim features,
// standardized) through `layers` ReLU layers of width `hidden` to `rank`
// coefficients alpha, and then through a linear layer of width out_dim (a
// rank-`rank` factor whose bias starts at the base solution) to a predicted
// primal-dual point z = (x, y) that seeds the solver.  Shapes are row-major
// with the batch as the leading dimension: Y[B x N] = X[B x K] W[K x N] + b.
//
// GEMMs: LDS-tiled kernels.
//   BF16 mode: operands rounded to bfloat16, products on MFMA
//     (v_mfma_f32_32x32x16_bf16, gfx950), FP32 accumulation: a 128x128 tile
//     per workgroup when the output has enough tiles to fill the GPU
//     (k_gemm_bf16_big), else a 64x64 tile with each wave64 owning a 32x32
//     quarter.
//   FP32 mode: the same tiling with FP32 FMA (every thread a 4x4 block); used
//     to check gradients against the FP64 reference at FP32 accuracy.
// Long reductions (dL/dalpha contracts over out_dim) are split over
// workgroups and the partial tiles are summed in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "host_util.h"
#include "lp.h"

namespace pdlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int GT = 64;   // output tile
constexpr int GK = 32;   // K per LDS stage

// element (r, c) of op(X) where op(X) is R x C; stored [R x C] (ld) or, when
// transposed, [C x R]
template <typename S, bool TR>
__device__ __forceinline__ float load_op(const S *X, int ld, int r, int c, int R, int Cc)
{
    if (r >= R || c >= Cc) return 0.0f;
    const size_t idx = TR ? (size_t)c * ld + r : (size_t)r * ld + c;
    if constexpr (sizeof(S) == 2) return bf2f(((const uint16_t *)X)[idx]);
    else return ((const float *)X)[idx];
}

// C (+ split offset) = op(A)[M x K] op(B)[K x N] over K range of this split;
// epilogue when splits == 1: + bias[N], ReLU, optional bf16 copy.
template <bool BF, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(const void *A, int lda, const void *B, int ldb, float *C, int ldc,
                                              int M, int N, int K, int kps, const float *bias, int relu,
                                              uint16_t *Cb)
{
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kb = blockIdx.z * kps, ke = min(K, kb + kps);
    float *Cout = C + (size_t)blockIdx.z * (size_t)M * ldc;
    const int t = threadIdx.x;
    if constexpr (BF) {
        // As[m][k], Bs[n][k]: k contiguous so each lane reads 8 bf16 at once
        __shared__ __attribute__((aligned(16))) uint16_t As[GT][GK + 8];
        __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GK + 8];
        const int wave = t >> 6, lane = t & 63;
        const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
        f32x16 acc;
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
        const uint16_t *Ah = (const uint16_t *)A, *Bh = (const uint16_t *)B;
        for (int k0 = kb; k0 < ke; k0 += GK) {
            for (int e = t; e < GT * GK; e += 256) {
                const int r = e / GK, c = e % GK;
                const int gr = m0 + r, gk = k0 + c;
                uint16_t va = 0, vb = 0;
                if (gr < M && gk < ke) va = Ah[TA ? (size_t)gk * lda + gr : (size_t)gr * lda + gk];
                const int gn = n0 + r;
                if (gn < N && gk < ke) vb = Bh[TB ? (size_t)gn * ldb + gk : (size_t)gk * ldb + gn];
                As[r][c] = va;
                Bs[r][c] = vb;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < GK; kk += 16) {
                bf16x8 a, b;
                const int kofs = kk + 8 * (lane >> 5);
                __builtin_memcpy(&a, &As[wm + (lane & 31)][kofs], 16);
                __builtin_memcpy(&b, &Bs[wn + (lane & 31)][kofs], 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
            }
            __syncthreads();
        }
        for (int v = 0; v < 16; ++v) {
            const int row = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int col = n0 + wn + (lane & 31);
            if (row < M && col < N) {
                float o = acc[v];
                if (gridDim.z == 1) {
                    if (bias) o += bias[col];
                    if (relu && o < 0.0f) o = 0.0f;
                    if (Cb) Cb[(size_t)row * ldc + col] = f2bf(o);
                }
                Cout[(size_t)row * ldc + col] = o;
            }
        }
    } else {
        __shared__ float As[GK][GT + 1];
        __shared__ float Bs[GK][GT + 1];
        const int tr = (t >> 4) * 4, tc = (t & 15) * 4;
        float acc[4][4] = {};
        for (int k0 = kb; k0 < ke; k0 += GK) {
            for (int e = t; e < GT * GK; e += 256) {
                const int r = e / GK, c = e % GK;
                const int gk = k0 + c;
                As[c][r] = gk < ke ? load_op<float, TA>((const float *)A, lda, m0 + r, gk, M, K) : 0.0f;
                Bs[c][r] = gk < ke ? load_op<float, !TB>((const float *)B, ldb, n0 + r, gk, N, K) : 0.0f;
            }
            __syncthreads();
            for (int kk = 0; kk < GK; ++kk) {
                float a[4], b[4];
                for (int i = 0; i < 4; ++i) {
                    a[i] = As[kk][tr + i];
                    b[i] = Bs[kk][tc + i];
                }
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
            }
            __syncthreads();
        }
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const int row = m0 + tr + i, col = n0 + tc + j;
                if (row < M && col < N) {
                    float o = acc[i][j];
                    if (gridDim.z == 1) {
                        if (bias) o += bias[col];
                        if (relu && o < 0.0f) o = 0.0f;
                        if (Cb) Cb[(size_t)row * ldc + col] = f2bf(o);
                    }
                    Cout[(size_t)row * ldc + col] = o;
                }
            }
    }
}

// BF16 GEMM for large outputs: a 128x128 tile per 256-thread workgroup,
// each wave64 owning 64x64 as 2x2 v_mfma_f32_32x32x16_bf16 tiles, K in
// stages of 64.  Operands are staged in LDS as [row][k] (k contiguous, rows
// padded to 72 so a wave's 16-byte operand reads hit distinct banks); a
// thread moves 16-byte vectors (8 bf16) and, for an operand stored with the
// other index contiguous, scatters each vector across 8 LDS rows.  The next
// stage's vectors are loaded into registers while the current one is
// multiplied.  Edges (and unaligned operands, vec == false) take guarded
// per-element loads with zero fill.  Same split and epilogue contract as
// k_gemm.
constexpr int BT = 128;   // output tile
constexpr int BK = 64;    // K per stage
constexpr int BP = 72;    // padded LDS row (bf16 elements): 144-byte rows put a wave's 16-byte reads on distinct banks
constexpr int BV = BT * BK / 8 / 256;   // 16-byte vectors per thread per operand and stage

// Vector v (0..BT*BK/8-1) of an operand's stage: rows r0.. of op(X) (R x Kdim),
// k in [k0, ke).  KC: stored with k contiguous (row-major in k); else the
// row index is contiguous.  Returns 8 bf16 in k order (KC) or in row order.
template <bool KC>
__device__ __forceinline__ uint4 stage_load(const uint16_t *X, int ld, int R, int r0, int k0, int ke, int v, bool vec)
{
    int r, k;
    if (KC) { r = v / (BK / 8); k = (v % (BK / 8)) * 8; }   // 128 rows x BK/8 vectors of k
    else { k = v % BK; r = (v / BK) * 8; }                   // 16 vectors of rows x BK k (k fastest: see stage_store)
    const int gr = r0 + r, gk = k0 + k;
    uint4 out;
    if (KC) {
        if (vec && gr < R && gk + 8 <= ke) return *(const uint4 *)(X + (size_t)gr * ld + gk);
        uint16_t e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (gr < R && gk + i < ke) ? X[(size_t)gr * ld + gk + i] : 0;
        __builtin_memcpy(&out, e, 16);
    } else {
        if (vec && gk < ke && gr + 8 <= R) return *(const uint4 *)(X + (size_t)gk * ld + gr);
        uint16_t e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (gk < ke && gr + i < R) ? X[(size_t)gk * ld + gr + i] : 0;
        __builtin_memcpy(&out, e, 16);
    }
    return out;
}

template <bool KC>
__device__ __forceinline__ void stage_store(uint16_t (*S)[BP], int v, uint4 val)
{
    if (KC) {
        *(uint4 *)&S[v / (BK / 8)][(v % (BK / 8)) * 8] = val;
    } else {
        // consecutive lanes take consecutive k, so each of the 8 scattered
        // 2-byte writes of a wave covers whole LDS rows rather than piling
        // onto a few banks
        uint16_t e[8];
        __builtin_memcpy(e, &val, 16);
        const int k = v % BK, r = (v / BK) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) S[r + i][k] = e[i];
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16_big(const uint16_t *A, int lda, const uint16_t *B, int ldb, float *C,
                                                       int ldc, int M, int N, int K, int kps, const float *bias,
                                                       int relu, uint16_t *Cb, int vec)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[BT][BP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BT][BP];
    const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
    const int kb = blockIdx.z * kps, ke = min(K, kb + kps);
    float *Cout = C + (size_t)blockIdx.z * (size_t)M * ldc;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // op(A) is M x K: stored [M][K] (k contiguous) unless TA; op(B)' is N x K:
    // stored [N][K] (k contiguous) when TB, else [K][N]
    constexpr bool AK = !TA, BKC = TB;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;
    uint4 ra[BV], rb[BV];
#pragma unroll
    for (int h = 0; h < BV; ++h) {
        ra[h] = stage_load<AK>(A, lda, M, m0, kb, ke, t + 256 * h, vec);
        rb[h] = stage_load<BKC>(B, ldb, N, n0, kb, ke, t + 256 * h, vec);
    }
    for (int k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
        for (int h = 0; h < BV; ++h) {
            stage_store<AK>(As, t + 256 * h, ra[h]);
            stage_store<BKC>(Bs, t + 256 * h, rb[h]);
        }
        __syncthreads();
        if (k0 + BK < ke) {
#pragma unroll
            for (int h = 0; h < BV; ++h) {
                ra[h] = stage_load<AK>(A, lda, M, m0, k0 + BK, ke, t + 256 * h, vec);
                rb[h] = stage_load<BKC>(B, ldb, N, n0, k0 + BK, ke, t + 256 * h, vec);
            }
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int kofs = kk + 8 * (lane >> 5);
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                __builtin_memcpy(&a[i], &As[wm + 32 * i + (lane & 31)][kofs], 16);
                __builtin_memcpy(&b[i], &Bs[wn + 32 * i + (lane & 31)][kofs], 16);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int col = n0 + wn + 32 * j + (lane & 31);
                if (row < M && col < N) {
                    float o = acc[i][j][v];
                    if (gridDim.z == 1) {
                        if (bias) o += bias[col];
                        if (relu && o < 0.0f) o = 0.0f;
                        if (Cb) Cb[(size_t)row * ldc + col] = f2bf(o);
                    }
                    Cout[(size_t)row * ldc + col] = o;
                }
            }
}

// C = sum over splits of the partial tiles, in split order
__global__ void k_split_sum(const float *part, int splits, int64_t len, float *C)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float s = part[i];
    for (int z = 1; z < splits; ++z) s += part[(size_t)z * len + i];
    C[i] = s;
}

__global__ void k_to_bf16(const float *x, uint16_t *y, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) y[i] = f2bf(x[i]);
}

// (x - mu) / sigma per feature; rows of width d
__global__ void k_standardize(const float *x, const float *mu, const float *sig, float *y, int64_t len, int d)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) y[i] = (x[i] - mu[i % d]) / sig[i % d];
}

// loss partials and dZ = 2 (Z - Z*) / (B * D)
__global__ void k_mse(const float *Z, const float *Zs, float *dZ, int64_t len, double *part)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < len) {
        const float d = Z[i] - Zs[i];
        s = (double)d * (double)d;
        dZ[i] = 2.0f * d / (float)len;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_parts(const double *part, int np, int64_t len, double *out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] / (double)len;
}

// column sums of a [rows x cols] matrix (bias gradients), rows in order
__global__ void k_colsum(const float *X, int rows, int cols, float *out)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
    out[c] = s;
}

// dH *= (H > 0)
__global__ void k_relu_back(float *dH, const float *H, int64_t len)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len && !(H[i] > 0.0f)) dH[i] = 0.0f;
}

__global__ void k_adam(float *p, float *m, float *v, const float *g, uint16_t *pb, int64_t len, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = f2bf(pi);
}

// out[b][s] = sum_j S[s][j] * D[b][j]   (S: CSR, rows x cols; D: [B x cols])
__global__ void k_sketch(const int *rp, const int *ci, const float *v, const float *D, int cols, float *out, int rows)
{
    const int s = blockIdx.x, b = blockIdx.y;
    double acc = 0.0;
    for (int p = rp[s] + threadIdx.x; p < rp[s + 1]; p += 256) acc += (double)v[p] * (double)D[(size_t)b * cols + ci[p]];
    __shared__ double sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)b * rows + s] = (float)sh[0];
}

inline int nblk(int64_t len) { return (int)((len + 255) / 256); }

// C = op(A) op(B) with optional epilogue; splits > 1 contracts K in parts
// (no epilogue then) through `scratch` (splits * M * N floats)
void gemm(hipStream_t st, bool bf, bool ta, bool tb, int M, int N, int K, const void *A, int lda, const void *B,
          int ldb, float *C, int ldc, const float *bias, bool relu, uint16_t *Cb, int splits, float *scratch)
{
    if (M <= 0 || N <= 0) return;
    if (splits < 1) splits = 1;
    const int kps = ((K + splits - 1) / splits + GK - 1) / GK * GK;
    splits = (K + kps - 1) / kps;
    if (splits < 1) splits = 1;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
    float *out = splits > 1 ? scratch : C;
    const int ldo = splits > 1 ? N : ldc;
    const int64_t big_tiles = (int64_t)((N + BT - 1) / BT) * ((M + BT - 1) / BT) * splits;
    if (bf && big_tiles >= 128) {
        // enough 128x128 tiles to fill the GPU: the large-tile MFMA kernel
        const bool vec = lda % 8 == 0 && ldb % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                         (reinterpret_cast<uintptr_t>(B) & 15) == 0;
        dim3 g2((N + BT - 1) / BT, (M + BT - 1) / BT, splits);
        const float *bs = splits > 1 ? nullptr : bias;
        const int rl = splits > 1 ? 0 : (int)relu;
        uint16_t *cb = splits > 1 ? nullptr : Cb;
        const uint16_t *Ah = (const uint16_t *)A, *Bh = (const uint16_t *)B;
        if (!ta && !tb) hipLaunchKernelGGL((k_gemm_bf16_big<false, false>), g2, dim3(256), 0, st, Ah, lda, Bh, ldb, out, ldo, M, N, K, kps, bs, rl, cb, (int)vec);
        else if (ta && !tb) hipLaunchKernelGGL((k_gemm_bf16_big<true, false>), g2, dim3(256), 0, st, Ah, lda, Bh, ldb, out, ldo, M, N, K, kps, bs, rl, cb, (int)vec);
        else if (!ta && tb) hipLaunchKernelGGL((k_gemm_bf16_big<false, true>), g2, dim3(256), 0, st, Ah, lda, Bh, ldb, out, ldo, M, N, K, kps, bs, rl, cb, (int)vec);
        else hipLaunchKernelGGL((k_gemm_bf16_big<true, true>), g2, dim3(256), 0, st, Ah, lda, Bh, ldb, out, ldo, M, N, K, kps, bs, rl, cb, (int)vec);
        if (splits > 1)
            hipLaunchKernelGGL(k_split_sum, dim3(nblk((int64_t)M * N)), dim3(256), 0, st, (const float *)scratch,
                               splits, (int64_t)M * N, C);
        HIPT(hipGetLastError());
        return;
    }
#define PDLP_GEMM_LAUNCH(BFV, TAV, TBV)                                                                            \
    hipLaunchKernelGGL((k_gemm<BFV, TAV, TBV>), grid, dim3(256), 0, st, A, lda, B, ldb, out, ldo, M, N, K, kps,     \
                       splits > 1 ? nullptr : bias, splits > 1 ? 0 : (int)relu, splits > 1 ? nullptr : Cb)
    if (bf) {
        if (!ta && !tb) PDLP_GEMM_LAUNCH(true, false, false);
        else if (ta && !tb) PDLP_GEMM_LAUNCH(true, true, false);
        else if (!ta && tb) PDLP_GEMM_LAUNCH(true, false, true);
        else PDLP_GEMM_LAUNCH(true, true, true);
    } else {
        if (!ta && !tb) PDLP_GEMM_LAUNCH(false, false, false);
        else if (ta && !tb) PDLP_GEMM_LAUNCH(false, true, false);
        else if (!ta && tb) PDLP_GEMM_LAUNCH(false, false, true);
        else PDLP_GEMM_LAUNCH(false, true, true);
    }
#undef PDLP_GEMM_LAUNCH
    if (splits > 1) {
        // splits > 1 is only used with ldc == N
        hipLaunchKernelGGL(k_split_sum, dim3(nblk((int64_t)M * N)), dim3(256), 0, st, (const float *)scratch, splits,
                           (int64_t)M * N, C);
    }
    HIPT(hipGetLastError());
}

}  // namespace pdlp

using namespace pdlp;

struct lpw_net {
    lpw_config cfg{};
    hipStream_t st = nullptr;
    Arena arena;
    int L = 0;                                   // linear layers = layers + 2
    std::vector<int> din, dout;                  // per layer
    std::vector<int64_t> woff, boff;             // offsets into the flat parameter vector
    int64_t nparam = 0;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;   // params, grads, Adam moments
    uint16_t *Pb = nullptr;                      // bf16 copy of the params
    float *mu = nullptr, *sig = nullptr;
    // activations for up to cfg.max_batch rows: A[0] = standardized input, A[l+1] = output of layer l
    std::vector<float *> Act, dAct;
    std::vector<uint16_t *> Actb, dActb;
    float *scratch = nullptr;
    int64_t scratch_len = 0;
    double *lpart = nullptr, *lout = nullptr;
    int64_t step = 0;
    std::string err;
};

namespace {

int net_fail(lpw_net *N, const HipError &h)
{
    char buf[512];
    snprintf(buf, sizeof(buf), "%s failed: %s", h.what, hipGetErrorString(h.e));
    if (N) N->err = buf;
    return h.e == hipErrorOutOfMemory ? LP_ERR_NOMEM : LP_ERR_HIP;
}

bool use_bf(const lpw_net *N) { return N->cfg.precision == LPW_BF16; }

// splits for the long contraction of layer l's input gradient
int splits_for(int K, int tiles)
{
    int s = 1;
    while (tiles * s < 512 && K / (s * 2) >= 256) s *= 2;
    return s;
}

void forward(lpw_net *N, const float *X, int B)
{
    hipStream_t st = N->st;
    const bool bf = use_bf(N);
    const int d0 = N->din[0];
    hipLaunchKernelGGL(k_standardize, dim3(nblk((int64_t)B * d0)), dim3(256), 0, st, X, (const float *)N->mu,
                       (const float *)N->sig, N->Act[0], (int64_t)B * d0, d0);
    if (bf)
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk((int64_t)B * d0)), dim3(256), 0, st, (const float *)N->Act[0],
                           N->Actb[0], (int64_t)B * d0);
    for (int l = 0; l < N->L; ++l) {
        const int K = N->din[l], Nn = N->dout[l];
        const bool relu = l < N->L - 2;
        const void *A = bf ? (const void *)N->Actb[l] : (const void *)N->Act[l];
        const void *W = bf ? (const void *)(N->Pb + N->woff[l]) : (const void *)(N->P + N->woff[l]);
        gemm(st, bf, false, false, B, Nn, K, A, K, W, Nn, N->Act[l + 1], Nn, N->P + N->boff[l], relu,
             bf ? N->Actb[l + 1] : nullptr, 1, nullptr);
    }
}

// backward from dZ (already in dAct[L]); fills G
void backward(lpw_net *N, int B)
{
    hipStream_t st = N->st;
    const bool bf = use_bf(N);
    for (int l = N->L - 1; l >= 0; --l) {
        const int K = N->din[l], Nn = N->dout[l];
        float *dY = N->dAct[l + 1];
        if (l < N->L - 2)   // ReLU layer: mask by the stored output
            hipLaunchKernelGGL(k_relu_back, dim3(nblk((int64_t)B * Nn)), dim3(256), 0, st, dY,
                               (const float *)N->Act[l + 1], (int64_t)B * Nn);
        if (bf)
            hipLaunchKernelGGL(k_to_bf16, dim3(nblk((int64_t)B * Nn)), dim3(256), 0, st, (const float *)dY,
                               N->dActb[l + 1], (int64_t)B * Nn);
        const void *dYo = bf ? (const void *)N->dActb[l + 1] : (const void *)dY;
        const void *Xo = bf ? (const void *)N->Actb[l] : (const void *)N->Act[l];
        // dW = X' dY  [K x Nn], contraction over the batch
        gemm(st, bf, true, false, K, Nn, B, Xo, K, dYo, Nn, N->G + N->woff[l], Nn, nullptr, false, nullptr, 1,
             nullptr);
        hipLaunchKernelGGL(k_colsum, dim3(nblk(Nn)), dim3(256), 0, st, (const float *)dY, B, Nn, N->G + N->boff[l]);
        if (l > 0) {
            // dX = dY W'  [B x K], contraction over Nn (long for the output layer)
            const void *Wo = bf ? (const void *)(N->Pb + N->woff[l]) : (const void *)(N->P + N->woff[l]);
            const int tiles = ((B + GT - 1) / GT) * ((K + GT - 1) / GT);
            int splits = splits_for(Nn, tiles);
            while (splits > 1 && (int64_t)splits * B * K > N->scratch_len) splits /= 2;
            gemm(st, bf, false, true, B, K, Nn, dYo, Nn, Wo, Nn, N->dAct[l], K, nullptr, false, nullptr, splits,
                 N->scratch);
        }
    }
}

}  // namespace

extern "C" {

void lpw_default_config(lpw_config *c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->in_dim = 256;
    c->hidden = 1024;
    c->layers = 3;
    c->rank = 64;
    c->out_dim = 0;
    c->max_batch = 256;
    c->precision = LPW_BF16;
    c->stream = nullptr;
}

int lpw_create(lpw_net **out, const lpw_config *cfg)
{
    if (!out || !cfg) return LP_ERR_ARG;
    *out = nullptr;
    if (cfg->in_dim <= 0 || cfg->hidden <= 0 || cfg->layers < 1 || cfg->rank <= 0 || cfg->out_dim <= 0 ||
        cfg->max_batch <= 0 || (cfg->precision != LPW_BF16 && cfg->precision != LPW_FP32))
        return LP_ERR_ARG;
    std::unique_ptr<lpw_net> N(new lpw_net());
    N->cfg = *cfg;
    N->st = (hipStream_t)cfg->stream;
    N->L = cfg->layers + 2;
    N->din.push_back(cfg->in_dim);
    for (int l = 0; l < cfg->layers; ++l) {
        N->dout.push_back(cfg->hidden);
        N->din.push_back(cfg->hidden);
    }
    N->dout.push_back(cfg->rank);
    N->din.push_back(cfg->rank);
    N->dout.push_back(cfg->out_dim);
    int64_t off = 0;
    for (int l = 0; l < N->L; ++l) {
        N->woff.push_back(off);
        off += (int64_t)N->din[l] * N->dout[l];
        N->boff.push_back(off);
        off += N->dout[l];
    }
    N->nparam = off;
    try {
        Arena &A = N->arena;
        N->P = A.make<float>(off);
        N->G = A.make<float>(off);
        N->Mm = A.make<float>(off);
        N->Vv = A.make<float>(off);
        N->Pb = A.make<uint16_t>(off);
        HIPT(hipMemsetAsync(N->Mm, 0, sizeof(float) * (size_t)off, N->st));
        HIPT(hipMemsetAsync(N->Vv, 0, sizeof(float) * (size_t)off, N->st));
        HIPT(hipMemsetAsync(N->G, 0, sizeof(float) * (size_t)off, N->st));
        N->mu = A.make<float>(cfg->in_dim);
        N->sig = A.make<float>(cfg->in_dim);
        std::vector<float> zeros(cfg->in_dim, 0.0f), ones(cfg->in_dim, 1.0f);
        h2d(N->st, N->mu, zeros.data(), cfg->in_dim);
        h2d(N->st, N->sig, ones.data(), cfg->in_dim);
        const int64_t Bm = cfg->max_batch;
        for (int l = 0; l <= N->L; ++l) {
            const int w = l == 0 ? N->din[0] : N->dout[l - 1];
            N->Act.push_back(A.make<float>(Bm * w));
            N->dAct.push_back(A.make<float>(Bm * w));
            N->Actb.push_back(A.make<uint16_t>(Bm * w));
            N->dActb.push_back(A.make<uint16_t>(Bm * w));
        }
        N->scratch_len = 64 * Bm * std::max(cfg->hidden, cfg->rank);
        N->scratch = A.make<float>(N->scratch_len);
        N->lpart = A.make<double>(nblk(Bm * (int64_t)cfg->out_dim));
        N->lout = A.make<double>(1);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N.get(), h);
    }
    *out = N.release();
    return LP_OK;
}

int64_t lpw_param_count(const lpw_net *N) { return N ? N->nparam : 0; }

int lpw_set_params(lpw_net *N, const float *host)
{
    if (!N || !host) return LP_ERR_ARG;
    try {
        h2d(N->st, N->P, host, N->nparam);
        hipLaunchKernelGGL(k_to_bf16, dim3(nblk(N->nparam)), dim3(256), 0, N->st, (const float *)N->P, N->Pb,
                           N->nparam);
        HIPT(hipMemsetAsync(N->Mm, 0, sizeof(float) * (size_t)N->nparam, N->st));
        HIPT(hipMemsetAsync(N->Vv, 0, sizeof(float) * (size_t)N->nparam, N->st));
        N->step = 0;
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_get_params(const lpw_net *Nc, float *host)
{
    lpw_net *N = const_cast<lpw_net *>(Nc);
    if (!N || !host) return LP_ERR_ARG;
    try {
        d2h(N->st, host, (const float *)N->P, N->nparam);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_set_norm(lpw_net *N, const float *mu, const float *sigma)
{
    if (!N || !mu || !sigma) return LP_ERR_ARG;
    for (int i = 0; i < N->cfg.in_dim; ++i)
        if (!(sigma[i] > 0.0f)) return LP_ERR_ARG;
    try {
        h2d(N->st, N->mu, mu, N->cfg.in_dim);
        h2d(N->st, N->sig, sigma, N->cfg.in_dim);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_forward(lpw_net *N, const float *X, int B, float *Z)
{
    if (!N || !X || !Z || B <= 0 || B > N->cfg.max_batch) return LP_ERR_ARG;
    try {
        forward(N, X, B);
        d2d(N->st, Z, (const float *)N->Act[N->L], (int64_t)B * N->cfg.out_dim);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_loss_grad(lpw_net *N, const float *X, const float *Zstar, int B, double *loss)
{
    if (!N || !X || !Zstar || B <= 0 || B > N->cfg.max_batch) return LP_ERR_ARG;
    try {
        forward(N, X, B);
        const int64_t len = (int64_t)B * N->cfg.out_dim;
        hipLaunchKernelGGL(k_mse, dim3(nblk(len)), dim3(256), 0, N->st, (const float *)N->Act[N->L], Zstar,
                           N->dAct[N->L], len, N->lpart);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, N->st, (const double *)N->lpart, nblk(len), len,
                           N->lout);
        backward(N, B);
        if (loss) d2h(N->st, loss, (const double *)N->lout, 1);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_get_grads(const lpw_net *Nc, float *host)
{
    lpw_net *N = const_cast<lpw_net *>(Nc);
    if (!N || !host) return LP_ERR_ARG;
    try {
        d2h(N->st, host, (const float *)N->G, N->nparam);
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_adam_step(lpw_net *N, float lr, float beta1, float beta2, float eps)
{
    if (!N || !(lr > 0.0f)) return LP_ERR_ARG;
    try {
        N->step += 1;
        const float c1 = 1.0f - std::pow(beta1, (float)N->step), c2 = 1.0f - std::pow(beta2, (float)N->step);
        hipLaunchKernelGGL(k_adam, dim3(nblk(N->nparam)), dim3(256), 0, N->st, N->P, N->Mm, N->Vv, (const float *)N->G,
                           N->Pb, N->nparam, lr, beta1, beta2, eps, c1, c2);
        HIPT(hipGetLastError());
        HIPT(hipStreamSynchronize(N->st));
    } catch (const HipError &h) {
        return net_fail(N, h);
    }
    return LP_OK;
}

int lpw_train_step(lpw_net *N, const float *X, const float *Zstar, int B, float lr, double *loss)
{
    const int rc = lpw_loss_grad(N, X, Zstar, B, loss);
    if (rc != LP_OK) return rc;
    return lpw_adam_step(N, lr, 0.9f, 0.999f, 1e-8f);
}

int lpw_gemm(int precision, int trans_a, int trans_b, int M, int N, int K, const void *A, int lda, const void *B,
             int ldb, float *C, int ldc, void *stream)
{
    if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0) return LP_ERR_ARG;
    try {
        gemm((hipStream_t)stream, precision == LPW_BF16, trans_a != 0, trans_b != 0, M, N, K, A, lda, B, ldb, C, ldc,
             nullptr, false, nullptr, 1, nullptr);
        HIPT(hipStreamSynchronize((hipStream_t)stream));
    } catch (const HipError &) {
        return LP_ERR_HIP;
    }
    return LP_OK;
}

int lpw_sketch(const int *rp, const int *ci, const float *v, int rows, const float *D, int cols, int B, float *out,
               void *stream)
{
    if (!rp || !ci || !v || !D || !out || rows <= 0 || cols <= 0 || B <= 0) return LP_ERR_ARG;
    try {
        hipLaunchKernelGGL(k_sketch, dim3(rows, B), dim3(256), 0, (hipStream_t)stream, rp, ci, v, D, cols, out, rows);
        HIPT(hipGetLastError());
        HIPT(hipStreamSynchronize((hipStream_t)stream));
    } catch (const HipError &) {
        return LP_ERR_HIP;
    }
    return LP_OK;
}

void lpw_free(lpw_net *N)
{
    if (!N) return;
    (void)hipStreamSynchronize(N->st);
    delete N;
}

const char *lpw_last_error(const lpw_net *N) { return N ? N->err.c_str() : ""; }

}  // extern "C"
