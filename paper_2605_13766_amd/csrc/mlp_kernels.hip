// mlp_kernels.hip -- gfx950 kernels of the surrogate's per-element MLP:
// a tiled BF16 MFMA GEMM (v_mfma_f32_16x16x32_bf16, FP32 accumulate) with
// fused epilogues (the bias gradient rides in the weight-gradient GEMM), the
// MSE gradient and Adam.
//
// Network: F_in -> 256 -> 256 -> 256 -> 12 (padded to 16 columns), SiLU after
// the first three layers, BF16 weights and activations, FP32 bias, FP32
// pre-activations kept for the backward pass.
#include "mlp_internal.h"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>

namespace mlpk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float to_f(__bf16 x) { return (float)x; }
__device__ inline float to_f(float x) { return x; }

// SiLU z sigma(z) with the hardware reciprocal (1 ulp) instead of an IEEE
// division: the result is rounded to BF16 right after
__device__ inline float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float dsilu_f(float z)
{
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

}  // namespace

// Stage a 64 (rows) x 64 (k) operand tile into S[row][k] as BF16.  The source
// is src[row][k] (k contiguous) or, when TRANS, src[k][row] (rows contiguous);
// each thread moves one 16-element run with 16-byte loads (two for BF16, four
// for FP32 sources), written to LDS as two 16-byte stores (k contiguous) or
// sixteen 2-byte stores (transposing).  Rows >= nrows and k outside [k0, ke)
// read as zero; row `ones` (if in [0, nrows)) reads as one for every k in
// [k0, ke) and is not loaded.
template <bool TRANS, typename TS, int LDK>
__device__ inline void stage_tile(__bf16 (*S)[LDK], const TS *src, int64_t ld, int row0, int nrows, int k0, int ke,
                                  int t, int ones)
{
    __bf16 v[16];
    const int a = t >> 2, b = (t & 3) * 16;   // direct: a = row, b = k offset; transposed: a = k, b = row offset
    const int row = TRANS ? row0 + b : row0 + a;
    const int k = TRANS ? k0 + a : k0 + b;
    const bool full = TRANS ? (k < ke && row + 16 <= nrows && (ones < row || ones >= row + 16))
                            : (row < nrows && row != ones && k + 16 <= ke);
    if (full) {
        const TS *p = TRANS ? src + (int64_t)k * ld + row : src + (int64_t)row * ld + k;
        if constexpr (sizeof(TS) == 2) {
            const uint4 u0 = reinterpret_cast<const uint4 *>(p)[0], u1 = reinterpret_cast<const uint4 *>(p)[1];
            const bf16x8 h0 = __builtin_bit_cast(bf16x8, u0), h1 = __builtin_bit_cast(bf16x8, u1);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                v[j] = h0[j];
                v[8 + j] = h1[j];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 f = reinterpret_cast<const float4 *>(p)[q];
                v[4 * q] = (__bf16)f.x;
                v[4 * q + 1] = (__bf16)f.y;
                v[4 * q + 2] = (__bf16)f.z;
                v[4 * q + 3] = (__bf16)f.w;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int rj = TRANS ? row + j : row, kj = TRANS ? k : k + j;
            const bool in_k = kj >= k0 && kj < ke;
            v[j] = (__bf16)(rj == ones ? (in_k ? 1.f : 0.f)
                            : rj < nrows && in_k ? to_f(src[TRANS ? (int64_t)kj * ld + rj : (int64_t)rj * ld + kj])
                                                 : 0.f);
        }
    }
    if constexpr (TRANS) {
#pragma unroll
        for (int j = 0; j < 16; ++j) S[b + j][a] = v[j];
    } else {
        uint4 *o = reinterpret_cast<uint4 *>(&S[a][b]);
        o[0] = __builtin_bit_cast(uint4, *reinterpret_cast<const bf16x8 *>(&v[0]));
        o[1] = __builtin_bit_cast(uint4, *reinterpret_cast<const bf16x8 *>(&v[8]));
    }
}

// C[M x N] = A[M x K] * B[K x N] with A stored [M][K] (or [K][M] when AT) and
// B stored [K][N] (or [N][K] when BT); inputs of type TA / TB are rounded to
// BF16 when staged in LDS.  One 256-thread workgroup computes a 64 x 64 tile,
// each wave a 32 x 32 quarter as 2 x 2 MFMA blocks; K advances 64 per stage
// (two MFMA k-steps).  Edges in M, N and K are zero-filled on load and masked
// on store.  Leading dimensions and base pointers must allow 16-byte loads of
// 16-element runs (multiples of 8 elements for BF16, 4 for FP32).
template <bool AT, bool BT, typename TA, typename TB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmArgs g)
{
    constexpr int BM = 64, BN = 64, BK = 64, LDK = BK + 8;
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][LDK];   // [m][k]
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][LDK];   // [n][k]
    const TA *A = (const TA *)g.A;
    const TB *B = (const TB *)g.B;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    // split reduction: z-slice blockIdx.z covers k in [kb, ke) and writes its own partial C
    const int kb = g.kchunk > 0 ? blockIdx.z * g.kchunk : 0;
    const int ke = g.kchunk > 0 ? min(g.K, kb + g.kchunk) : g.K;
    float *const Cz = g.C + (int64_t)blockIdx.z * g.zstride;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int q = lane >> 4, c = lane & 15;
    for (int k0 = kb; k0 < ke; k0 += BK) {
        // A: rows m, stored [M][K] (k contiguous) or [K][M] (m contiguous)
        stage_tile<AT, TA, LDK>(As, A, g.lda, m0, g.M, k0, ke, t, g.ones_row);
        // B: rows n, stored [N][K] (k contiguous) when BT, else [K][N] (n contiguous)
        stage_tile<!BT, TB, LDK>(Bs, B, g.ldb, n0, g.N, k0, ke, t, -1);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + c][kk + 8 * q]);
                bfr[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * i + c][kk + 8 * q]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // ---- epilogue: lane holds rows 4*(lane/16)+r, column lane%16 of each block
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * q + r;
                const int n = n0 + wn + 16 * j + c;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const int64_t o = (int64_t)m * g.ldc + n;
                if (EPI == EPI_STORE) {
                    Cz[o] = v;
                } else if (EPI == EPI_BIAS) {
                    g.C[o] = v + g.bias[n];
                } else if (EPI == EPI_BIAS_SILU) {
                    const float z = v + g.bias[n];
                    g.C[o] = z;                          // pre-activation, for backward
                    g.act[o] = (__bf16)silu_f(z);        // next layer's input
                } else if (EPI == EPI_DSILU) {
                    g.C[o] = v * dsilu_f(g.zsave[o]);    // dZ = dA * silu'(Z)
                }
            }
}

// dY = 2 * mask * (Y - T) / count for the first n_out columns (0 on padding),
// and per-block partial sums of mask * (Y - T)^2.
__global__ void mse_grad_kernel(const float *Y, const float *T, const float *mask, float *dY,
                                float *partial, int64_t M, int n_out, int ld, float inv_count)
{
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (i < M * ld) {
        const int64_t row = i / ld;
        const int col = (int)(i % ld);
        float d = 0.f;
        if (col < n_out) {
            const float mk = mask ? mask[row * n_out + col] : 1.f;
            const float e = Y[i] - T[row * n_out + col];
            d = 2.f * mk * e * inv_count;
            s = mk * e * e;
        }
        dY[i] = d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[0] = sum(partial[0..n)) * scale (one block).
__global__ void sum_kernel(const float *partial, int n, float scale, float *out)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// Adam (Kingma & Ba): m, v, w in FP32; bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t;
// wb (or NULL) receives the updated weight rounded to BF16.
__global__ void adam_kernel(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2, __bf16 *wb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (__bf16)wi;
}

// BF16 copies of the FP32 master weights.
__global__ void to_bf16_kernel(const float *src, __bf16 *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (__bf16)src[i];
}

// ------------------------------------------------------------------ launchers

template <bool AT, bool BT, typename TA, typename TB, int EPI>
static hipError_t launch_t(const GemmArgs &g, hipStream_t s, int splits = 1)
{
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    hipLaunchKernelGGL((gemm_kernel<AT, BT, TA, TB, EPI>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// out[i] = sum over z of part[z * stride + i], z ascending (deterministic);
// the loads of eight slices are issued before their additions
__global__ void sum_splits_kernel(const float *part, int splits, int64_t stride, int64_t n, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float acc = 0.f;
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * stride + i];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; z < splits; ++z) acc += part[(int64_t)z * stride + i];
    out[i] = acc;
}

hipError_t gemm_forward(const GemmArgs &g, int epi, hipStream_t s)
{
    // A = activations bf16 [M][K], B = W bf16 [K][N]
    switch (epi) {
    case EPI_BIAS_SILU: return launch_t<false, false, __bf16, __bf16, EPI_BIAS_SILU>(g, s);
    case EPI_BIAS: return launch_t<false, false, __bf16, __bf16, EPI_BIAS>(g, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gemm_backward_data(const GemmArgs &g, int epi, hipStream_t s)
{
    // C[M][K_l] = dZ f32 [M][N_l] * W^T, W bf16 stored [K_l][N_l] = [N_gemm][K_gemm]
    switch (epi) {
    case EPI_DSILU: return launch_t<false, true, float, __bf16, EPI_DSILU>(g, s);
    case EPI_STORE: return launch_t<false, true, float, __bf16, EPI_STORE>(g, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t gemm_backward_weight(const GemmArgs &g, float *work, int64_t work_floats, hipStream_t s)
{
    // C[K_l][N_l] = act^T * dZ: act bf16 stored [M][K_l] = [K_gemm][M_gemm], dZ f32 [M][N_l].
    // The output has few 64 x 64 tiles, so the long reduction (the minibatch) is split
    // into z-slices of at least 512 rows, at most about 512 workgroups in all; the
    // slices' partial products go to `work` and are summed in slice order.
    const int64_t tiles = (int64_t)((g.N + 63) / 64) * ((g.M + 63) / 64);
    const int64_t out_floats = (int64_t)g.M * g.ldc;
    int splits = (int)std::min<int64_t>({(512 + tiles - 1) / tiles, (g.K + 511) / 512,
                                         work ? work_floats / std::max<int64_t>(out_floats, 1) : 1});
    if (splits <= 1) return launch_t<true, false, __bf16, float, EPI_STORE>(g, s);
    GemmArgs a = g;
    a.kchunk = (int)((((int64_t)g.K + splits - 1) / splits + 31) / 32 * 32);
    splits = (int)(((int64_t)g.K + a.kchunk - 1) / a.kchunk);
    a.C = work;
    a.zstride = out_floats;
    hipError_t e = launch_t<true, false, __bf16, float, EPI_STORE>(a, s, splits);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_splits_kernel, dim3((unsigned)((out_floats + 255) / 256)), dim3(256), 0, s, work, splits,
                       out_floats, out_floats, g.C);
    return hipGetLastError();
}

hipError_t mse_grad(const float *Y, const float *T, const float *mask, float *dY, float *partial,
                    int64_t M, int n_out, int ld, hipStream_t s)
{
    const int64_t n = M * ld;
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks), dim3(256), 0, s, Y, T, mask, dY, partial, M, n_out, ld,
                       1.0f / (float)(M * n_out));
    return hipGetLastError();
}

int mse_partials(int64_t M, int ld) { return (int)((M * ld + 255) / 256); }

hipError_t sum_partials(const float *partial, int n, float scale, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, partial, n, scale, out);
    return hipGetLastError();
}

hipError_t adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                float eps, int64_t t, __bf16 *wb, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, n, lr, b1,
                       b2, eps, c1, c2, wb);
    return hipGetLastError();
}

hipError_t to_bf16(const float *src, __bf16 *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace mlpk
