// Private declarations of the surrogate data-path kernels
// (surrogate_kernels.hip) used by surrogate.cpp.  Not part of the boundary.
#pragma once

#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace surk {

constexpr int N_FEAT = 96;
constexpr int N_OUT = 12;

// per-rod feature constants
enum RodFeat { RF_LOGE, RF_RADIUS, RF_SQRT_RHOA_EI, RF_ALPHA, RF_CLAMP0, RF_AMP, RF_FREQ, RF_PHASE, NRF };
constexpr float AMP_SCALE = 1e-5f;   // couple amplitude unit of the features (N m/m)

struct WinArgs {
    rodk::DevBatch<float> B;     // FP32 batch (edge form), state at time `time`
    const int32_t *win_rod;      // [n_windows]
    const int64_t *win_first;    // [R] first window of each rod
    const float *rodf;           // [R][NRF]
    int64_t n_windows;
    float tau;                   // k dt
    double time;
    float2 *phase;               // [R] scratch: sin and cos of each rod's couple phase at `time`
};

// raw FP32 rows and/or BF16 rows (x - mu) * isd (isd = 1 / sd per column)
hipError_t features(const WinArgs &A, float *raw, __bf16 *xn, const float *mu, const float *isd, hipStream_t s);
hipError_t targets(const WinArgs &A, const rodk::DevBatch<float> &S0, float *tgt, float *mask, hipStream_t s);
// n_max: the longest rod (<= 512: one workgroup per rod; else two passes)
hipError_t apply(const WinArgs &A, const float *y, int ldy, const float *mu, const float *sd, const int32_t *skip,
                 float *disp, const int32_t *elem_rod, const int64_t *elem_first, int64_t n_elems, hipStream_t s,
                 int n_max = 0);
hipError_t gather_rows(const float *fraw, const float *traw, const float *mraw, const int64_t *idx, int64_t rows,
                       const float *mu_x, const float *isd_x, const float *mu_t, const float *sd_t, __bf16 *x, float *t,
                       float *m, hipStream_t s);
// dst rod k <-> src rod map[k] (to_src: copy back into src); sel[k] == 0 skips k
hipError_t copy_rods(const rodk::DevBatch<float> &dst, const rodk::DevBatch<float> &src, const int32_t *map,
                     const int32_t *sel, int n_map, int n, bool state_only, bool to_src, hipStream_t s);
// seeded perturbation of the free state (positions, velocities, frames, omega), in place
hipError_t perturb(const rodk::DevBatch<float> &B, const int32_t *elem_rod, const int64_t *elem_first, int64_t n_elems,
                   const float noise[4], float tau, uint64_t seed, hipStream_t s);
hipError_t colstats(const float *a, const float *mask, int64_t rows, int cols, double *out, hipStream_t s);
hipError_t judge_errors(const rodk::DevBatch<float> &main, const rodk::DevBatch<float> &ref, const int32_t *map,
                        int n_map, float *err, hipStream_t s);

}  // namespace surk
