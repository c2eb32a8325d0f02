// Private declarations of the surrogate MLP kernels (mlp_kernels.hip) used by
// the host runtime (surrogate.cpp).  Not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mlpk {

enum Epilogue { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_DSILU = 3 };

struct GemmArgs {
    const void *A;          // see the launcher for layout and type
    const void *B;
    int64_t lda, ldb, ldc;
    int M, N, K;
    float *C;               // FP32 output (pre-activation, dZ or plain product)
    const float *bias;      // [N] for EPI_BIAS / EPI_BIAS_SILU
    __bf16 *act;            // [M][ldc] BF16 SiLU output for EPI_BIAS_SILU
    const float *zsave;     // [M][ldc] pre-activation for EPI_DSILU
    int kchunk = 0;         // split reduction: K per z-slice (0: one slice)
    int64_t zstride = 0;    // offset between the slices' outputs
    int ones_row = -1;      // row of A (in [0, M)) that reads as all ones: with A^T dZ
                            // it makes that row of C the column sums of dZ (a bias gradient)
};

hipError_t gemm_forward(const GemmArgs &g, int epi, hipStream_t s);
hipError_t gemm_backward_data(const GemmArgs &g, int epi, hipStream_t s);
// work: scratch of work_floats floats for the split reduction (NULL: no split).
// With g.ones_row = K_l and g.M = K_l + 1, row K_l of C is the bias gradient.
hipError_t gemm_backward_weight(const GemmArgs &g, float *work, int64_t work_floats, hipStream_t s);
hipError_t mse_grad(const float *Y, const float *T, const float *mask, float *dY, float *partial,
                    int64_t M, int n_out, int ld, hipStream_t s);
int mse_partials(int64_t M, int ld);
hipError_t sum_partials(const float *partial, int n, float scale, float *out, hipStream_t s);
// wb: BF16 copies of the updated weights (NULL: none)
hipError_t adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                float eps, int64_t t, __bf16 *wb, hipStream_t s);
hipError_t to_bf16(const float *src, __bf16 *dst, int64_t n, hipStream_t s);

// Fused inference (mlp_infer.hip).  Weights are first packed from the BF16
// internal layout (layer l at w_offset[l], [K][ld[l]] row-major) into MFMA
// fragments (infer_fragments_bytes() bytes, 16-byte aligned).
struct PackArgs {
    int64_t w_offset[4];
    int ld[4];
};
struct InferArgs {
    const __bf16 *x;        // [M][96] standardised inputs, rows 16-byte aligned
    int64_t M;
    const __bf16 *frag;     // packed fragments
    const float *bias[4];   // FP32 biases (256, 256, 256, 16 values)
    float *y;               // [M][ldy] outputs, ldy 16 (all 16 columns) or 12
    int ldy;
};
int infer_fragments_bytes();
hipError_t pack_fragments(const __bf16 *wb, const PackArgs &p, __bf16 *frags, hipStream_t s);
hipError_t mlp_infer(const InferArgs &a, hipStream_t s);

}  // namespace mlpk
