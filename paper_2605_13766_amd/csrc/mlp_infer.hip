// mlp_infer.hip -- fused inference of the surrogate MLP on gfx950: all four
// layers of a 64-row block in one wave, activations never leaving registers.
//
// Each layer is computed transposed, Z^T = W^T H^T, with
// v_mfma_f32_16x16x32_bf16: the weights are the A operand (16 outputs x 32
// inputs), the activations the B operand (32 inputs x 16 rows).  In that
// instruction lane l (g = l / 16, i = l % 16) holds A[i][8g + j], B[8g + j][i]
// (j = 0..7) and D[4g + r][i] (r = 0..3).  The output tiles 2c and 2c + 1 of
// one layer therefore leave lane l with outputs 32c + 4g + r and
// 32c + 16 + 4g + r of row i: exactly one B operand of the next layer's input
// chunk c, once that layer's input order inside the chunk is permuted to
// slot 8g + j <-> input 32c + (j < 4 ? 4g + j : 12 + 4g + j).  The permutation
// is folded into the weight packing, so bias, SiLU and the BF16 rounding are
// applied in registers and the next layer starts at once.
//
// Weights are packed once per update into 1 KB fragments (one per output tile
// and input chunk, lane-major, 16 bytes per lane) read straight from L2 with
// one 128-bit load per lane; each fragment feeds IR MFMAs (the wave's 16-row
// blocks), and fragments are fetched two tiles ahead of their use.
#include "mlp_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mlpk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Row blocks per wave and waves per SIMD, measured on 17M rows once the SiLU
// uses the hardware reciprocal: 4 blocks (64 rows) at 1 wave per SIMD 6.04 ms,
// 3 at 1 wave 6.25 ms, 2 at 2 waves 6.51 ms, 1 at 4 waves 15.3 ms.  With the
// lighter epilogue the weight reuse of 64 rows per fragment wins.
#ifndef ROD_MLP_ROW_BLOCKS
#define ROD_MLP_ROW_BLOCKS 4
#endif
#ifndef ROD_MLP_WAVES_PER_SIMD
#define ROD_MLP_WAVES_PER_SIMD 1
#endif
constexpr int IR = ROD_MLP_ROW_BLOCKS;                 // 16-row blocks per wave
constexpr int ROWS_PER_WAVE = 16 * IR;
constexpr int WAVES = 4;
// per layer: 32-wide input chunks 3, 8, 8, 8; 16-wide output tiles 16, 16, 16, 1;
// fragments (tile-major, then chunk) start at 0, 48, 176, 304
constexpr int F_BASE[4] = {0, 48, 176, 304};
constexpr int N_FRAG = 312;

// SiLU z sigma(z) with the hardware reciprocal (1 ulp) instead of an IEEE
// division: the result is rounded to BF16 right after
__device__ inline float silu_f(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

// input k of layer l stored in slot (c, g, j) of its B operand
__host__ __device__ inline int input_of_slot(int l, int c, int g, int j)
{
    if (l == 0) return 32 * c + 8 * g + j;
    return 32 * c + (j < 4 ? 4 * g + j : 12 + 4 * g + j);
}

template <int CI>
__device__ __forceinline__ void load_tile(uint4 (&w)[CI], const uint4 *__restrict__ frag, int t, int lane)
{
#pragma unroll
    for (int c = 0; c < CI; ++c) w[c] = frag[(t * CI + c) * 64 + lane];
}

// acc = bias + W^T hin for one output tile (the accumulators start at the bias)
template <int CI>
__device__ __forceinline__ void mma_tile(f32x4 (&acc)[IR], const uint4 (&w)[CI], const bf16x8 (&hin)[IR][CI],
                                         const float *__restrict__ bias, int t, int g)
{
    const float4 b = *reinterpret_cast<const float4 *>(bias + 16 * t + 4 * g);
#pragma unroll
    for (int q = 0; q < IR; ++q) acc[q] = f32x4{b.x, b.y, b.z, b.w};
#pragma unroll
    for (int c = 0; c < CI; ++c) {
        const bf16x8 a = as_bf16x8(w[c]);
#pragma unroll
        for (int q = 0; q < IR; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hin[q][c], acc[q], 0, 0, 0);
    }
}

template <int TO>
__device__ __forceinline__ void epilogue(const f32x4 (&acc)[IR], bf16x8 (&hout)[IR][TO / 2], int t)
{
#pragma unroll
    for (int q = 0; q < IR; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) hout[q][t >> 1][(t & 1) * 4 + r] = (__bf16)silu_f(acc[q][r]);
}

// One hidden layer: hout = bf16(silu(W^T hin + b)) for the wave's IR row blocks,
// software-pipelined: the MFMAs of tile t + 1 are issued before the SiLU
// epilogue of tile t, so the vector ALU works in the matrix cores' shadow;
// fragments are fetched two tiles ahead.
template <int CI, int TO>
__device__ __forceinline__ void dense_silu(const bf16x8 (&hin)[IR][CI], bf16x8 (&hout)[IR][TO / 2],
                                           const uint4 *__restrict__ frag, const float *__restrict__ bias, int lane)
{
    const int g = lane >> 4;
    uint4 w0[CI], w1[CI];
    f32x4 acc0[IR], acc1[IR];
    load_tile<CI>(w0, frag, 0, lane);
    load_tile<CI>(w1, frag, 1, lane);
    mma_tile<CI>(acc0, w0, hin, bias, 0, g);
#pragma unroll
    for (int t = 0; t < TO; t += 2) {
        // acc0 holds tile t; w1 holds tile t + 1
        if (t + 2 < TO) load_tile<CI>(w0, frag, t + 2, lane);
        mma_tile<CI>(acc1, w1, hin, bias, t + 1, g);
        epilogue<TO>(acc0, hout, t);
        if (t + 3 < TO) load_tile<CI>(w1, frag, t + 3, lane);
        if (t + 2 < TO) mma_tile<CI>(acc0, w0, hin, bias, t + 2, g);
        epilogue<TO>(acc1, hout, t + 1);
    }
}

__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(ROD_MLP_WAVES_PER_SIMD, ROD_MLP_WAVES_PER_SIMD)))
void mlp_infer_kernel(const InferArgs a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int64_t m0 = ((int64_t)blockIdx.x * WAVES + wave) * ROWS_PER_WAVE;
    if (m0 >= a.M) return;   // no barriers below: a wave with no rows leaves at once
    const uint4 *__restrict__ frag = reinterpret_cast<const uint4 *>(a.frag);
    bf16x8 x[IR][3];
#pragma unroll
    for (int q = 0; q < IR; ++q) {
        const int64_t row = m0 + 16 * q + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uint4 u = {0u, 0u, 0u, 0u};
            if (row < a.M) u = *reinterpret_cast<const uint4 *>(a.x + row * 96 + 32 * c + 8 * g);
            x[q][c] = as_bf16x8(u);
        }
    }
    bf16x8 h1[IR][8], h2[IR][8];
    dense_silu<3, 16>(x, h1, frag + F_BASE[0] * 64, a.bias[0], lane);
    dense_silu<8, 16>(h1, h2, frag + F_BASE[1] * 64, a.bias[1], lane);
    dense_silu<8, 16>(h2, h1, frag + F_BASE[2] * 64, a.bias[2], lane);
    // output layer: one 16-wide tile (12 outputs and 4 zero columns), no activation
    const float4 b = *reinterpret_cast<const float4 *>(a.bias[3] + 4 * g);
    f32x4 acc[IR];
#pragma unroll
    for (int q = 0; q < IR; ++q) acc[q] = f32x4{b.x, b.y, b.z, b.w};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const bf16x8 w = as_bf16x8(frag[(F_BASE[3] + c) * 64 + lane]);
#pragma unroll
        for (int q = 0; q < IR; ++q) acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, h1[q][c], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < IR; ++q) {
        const int64_t row = m0 + 16 * q + i;
        if (row >= a.M) continue;
        const float4 o{acc[q][0], acc[q][1], acc[q][2], acc[q][3]};
        if (a.ldy == 16) {
            *reinterpret_cast<float4 *>(a.y + row * 16 + 4 * g) = o;
        } else if (g < 3) {
            float *p = a.y + row * a.ldy + 4 * g;
            p[0] = o.x; p[1] = o.y; p[2] = o.z; p[3] = o.w;
        }
    }
}

// fragment f of layer l, lane (g, i): W_l[input_of_slot(l, c, g, j)][16 t + i], j = 0..7
__global__ void pack_fragments_kernel(const __bf16 *wb, PackArgs p, __bf16 *frags)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= N_FRAG * 64) return;
    const int f = gid >> 6, lane = gid & 63, g = lane >> 4, i = lane & 15;
    const int l = f < 48 ? 0 : f < 176 ? 1 : f < 304 ? 2 : 3;
    const int base = l == 0 ? 0 : l == 1 ? 48 : l == 2 ? 176 : 304;
    const int chunks = l == 0 ? 3 : 8;
    const int fl = f - base, t = fl / chunks, c = fl % chunks;
    const __bf16 *W = wb + p.w_offset[l];
    const int ld = p.ld[l];
    __bf16 *o = frags + (int64_t)gid * 8;
    for (int j = 0; j < 8; ++j) o[j] = W[(int64_t)input_of_slot(l, c, g, j) * ld + 16 * t + i];
}

}  // namespace

int infer_fragments_bytes() { return N_FRAG * 1024; }

hipError_t pack_fragments(const __bf16 *wb, const PackArgs &p, __bf16 *frags, hipStream_t s)
{
    hipLaunchKernelGGL(pack_fragments_kernel, dim3((N_FRAG * 64 + 255) / 256), dim3(256), 0, s, wb, p, frags);
    return hipGetLastError();
}

hipError_t mlp_infer(const InferArgs &a, hipStream_t s)
{
    if (a.M <= 0) return hipSuccess;
    if (a.ldy != 16 && a.ldy != 12) return hipErrorInvalidValue;
    const int64_t per_block = (int64_t)WAVES * ROWS_PER_WAVE;
    const int64_t blocks = (a.M + per_block - 1) / per_block;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)blocks), dim3(64 * WAVES), 0, s, a);
    return hipGetLastError();
}

}  // namespace mlpk
