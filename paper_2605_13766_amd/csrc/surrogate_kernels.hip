// surrogate_kernels.hip -- gfx950 kernels of the learned coarse step's data
// path on FP32 rod batches (edge form: per element the edge r_{i+1} - r_i,
// per rod node 0 in the tail position fields):
//   window features (5-element stencil in the centre element's frame),
//   training targets (change of the target node and element over tau = k dt),
//   applying predicted deltas (two phases: node displacements, then edges and
//   directors), minibatch gathering, rod copies for the judge, and the judge's
//   per-rod error measures.
// One thread per window, element or rod; neighbours are read from the slot
// arrays (adjacent slots of the same tile).
#include "rod.h"
#include "surrogate_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace surk {

using rodk::DevBatch;

namespace {

struct V3 {
    float x, y, z;
};
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }

struct Rod {
    const DevBatch<float> &B;
    int r;
    int64_t s0;   // slot of element 0
    int n;
    __device__ Rod(const DevBatch<float> &b, int rod) : B(b), r(rod), s0(b.rod_slot[rod]), n(b.rod_n[rod]) {}
    __device__ float st(int f, int i) const { return B.state[(int64_t)f * B.n_slots + s0 + i]; }
    __device__ V3 edge(int i) const { return {st(rodk::RX, i), st(rodk::RY, i), st(rodk::RZ, i)}; }
    __device__ V3 node_v(int j) const
    {
        if (j < n) return {st(rodk::VX, j), st(rodk::VY, j), st(rodk::VZ, j)};
        return {B.tail[rodk::TVX * B.n_rods + r], B.tail[rodk::TVY * B.n_rods + r], B.tail[rodk::TVZ * B.n_rods + r]};
    }
    __device__ V3 anchor() const
    {
        return {B.tail[rodk::TRX * B.n_rods + r], B.tail[rodk::TRY * B.n_rods + r], B.tail[rodk::TRZ * B.n_rods + r]};
    }
    __device__ V3 omega(int i) const { return {st(rodk::WX, i), st(rodk::WY, i), st(rodk::WZ, i)}; }
    __device__ void dirs(int i, float q[9]) const
    {
        for (int k = 0; k < 9; ++k) q[k] = st(rodk::Q00 + k, i);
    }
    __device__ float lh(int i) const { return B.param[(int64_t)rodk::P_LH * B.n_slots + s0 + i]; }
};

__device__ inline V3 matvec(const float q[9], V3 v)
{
    return {q[0] * v.x + q[1] * v.y + q[2] * v.z, q[3] * v.x + q[4] * v.y + q[5] * v.z,
            q[6] * v.x + q[7] * v.y + q[8] * v.z};
}
__device__ inline V3 matTvec(const float q[9], V3 v)
{
    return {q[0] * v.x + q[3] * v.y + q[6] * v.z, q[1] * v.x + q[4] * v.y + q[7] * v.z,
            q[2] * v.x + q[5] * v.y + q[8] * v.z};
}

// midpoint of element j minus midpoint of element c, from the edges
__device__ inline V3 mid_offset(const Rod &R, int c, int j)
{
    if (j == c) return {0.f, 0.f, 0.f};
    if (j > c) {
        V3 s = 0.5f * R.edge(c);
        for (int m = c + 1; m < j; ++m) s = s + R.edge(m);
        return s + 0.5f * R.edge(j);
    }
    V3 s = 0.5f * R.edge(c);
    for (int m = j + 1; m < c; ++m) s = s + R.edge(m);
    s = s + 0.5f * R.edge(j);
    return {-s.x, -s.y, -s.z};
}

// rotation vector of qa qb^T (series for small angles, atan2 otherwise)
__device__ inline V3 log_rel(const float qa[9], const float qb[9])
{
    auto dot = [&](int a, int b) {
        return qa[3 * a] * qb[3 * b] + qa[3 * a + 1] * qb[3 * b + 1] + qa[3 * a + 2] * qb[3 * b + 2];
    };
    const float w0 = 0.5f * (dot(2, 1) - dot(1, 2));
    const float w1 = 0.5f * (dot(0, 2) - dot(2, 0));
    const float w2 = 0.5f * (dot(1, 0) - dot(0, 1));
    const float c = 0.5f * (dot(0, 0) + dot(1, 1) + dot(2, 2) - 1.0f);
    const float s2 = w0 * w0 + w1 * w1 + w2 * w2;
    float f;
    if (c > 0.f && s2 < 4e-3f)
        f = 1.f + s2 * (1.f / 6 + s2 * (3.f / 40 + s2 * (5.f / 112 + s2 * (35.f / 1152))));
    else {
        const float s = sqrtf(s2);
        f = s > 0.f ? atan2f(s, c) / s : 1.f;
    }
    return {f * w0, f * w1, f * w2};
}

// q <- exp([u]x) q
__device__ inline void rotate_left(float q[9], V3 u)
{
    const float x = u.x * u.x + u.y * u.y + u.z * u.z;
    float a, b;
    if (x < 1e-2f) {
        a = 1.f + x * (-1.f / 6 + x * (1.f / 120 + x * (-1.f / 5040)));
        b = 0.5f + x * (-1.f / 24 + x * (1.f / 720 + x * (-1.f / 40320)));
    } else {
        const float t = sqrtf(x);
        a = sinf(t) / t;
        b = (1.f - cosf(t)) / x;
    }
    for (int j = 0; j < 3; ++j) {
        const float c0 = q[j], c1 = q[3 + j], c2 = q[6 + j];
        const float k0 = u.y * c2 - u.z * c1, k1 = u.z * c0 - u.x * c2, k2 = u.x * c1 - u.y * c0;
        const float kk0 = u.y * k2 - u.z * k1, kk1 = u.z * k0 - u.x * k2, kk2 = u.x * k1 - u.y * k0;
        q[j] = c0 + a * k0 + b * kk0;
        q[3 + j] = c1 + a * k1 + b * kk1;
        q[6 + j] = c2 + a * k2 + b * kk2;
    }
}

}  // namespace

// ---------------------------------------------------------------- features
// sin and cos of each rod's couple phase 2 pi f t + phi, once per rod (FP64)
__global__ void phase_kernel(const float *rodf, int n_rods, double time, float2 *out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rods) return;
    const float *rf = rodf + (int64_t)r * NRF;
    const double ph = 2.0 * M_PI * (double)rf[RF_FREQ] * time + (double)rf[RF_PHASE];
    out[r] = float2{(float)sin(ph), (float)cos(ph)};
}

// midpoint of element c + D minus midpoint of element c (D = -2..2), from the
// edges, in the order of mid_offset
template <int D>
__device__ inline V3 mid_off(const Rod &R, int c)
{
    if constexpr (D == 0) {
        return {0.f, 0.f, 0.f};
    } else if constexpr (D > 0) {
        V3 s = 0.5f * R.edge(c);
        if constexpr (D == 2) s = s + R.edge(c + 1);
        return s + 0.5f * R.edge(c + D);
    } else {
        V3 s = 0.5f * R.edge(c);
        if constexpr (D == -2) s = s + R.edge(c - 1);
        s = s + 0.5f * R.edge(c + D);
        return {-s.x, -s.y, -s.z};
    }
}

// Write 16 feature values at columns col0..col0+15 of window g: FP32 rows
// and/or BF16 rows standardised as (x - mu) * (1 / sd), as 16-byte stores.
__device__ inline void emit16(const float (&v)[16], int col0, int64_t g, float *raw, __bf16 *xn, const float *mu,
                              const float *isd)
{
    if (raw) {
        float4 *o = reinterpret_cast<float4 *>(raw + g * N_FEAT + col0);
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = float4{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
    }
    if (xn) {
        // xn points at this thread's BF16 row (in LDS: the wave's staging tile)
        uint4 *o = reinterpret_cast<uint4 *>(xn + col0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            __bf16 b[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) b[j] = (__bf16)((v[8 * k + j] - mu[col0 + 8 * k + j]) * isd[col0 + 8 * k + j]);
            o[k] = __builtin_bit_cast(uint4, b);
        }
    }
}

// stencil slot D (element c + D) of window g
template <int D>
__device__ inline void emit_slot(const Rod &R, int c, int n, const float (&qc)[9], V3 uc, float iL, float tau,
                                 int64_t g, float *raw, __bf16 *xn, const float *mu, const float *isd)
{
    float o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) o[k] = 0.f;
    const int j = c + D;
    if (j >= 0 && j < n) {
        const V3 d = matvec(qc, mid_off<D>(R, c));
        o[0] = d.x * iL; o[1] = d.y * iL; o[2] = d.z * iL;
        const V3 uj = 0.5f * (R.node_v(j) + R.node_v(j + 1));
        const V3 du = matvec(qc, uj - uc);
        o[3] = du.x * tau * iL; o[4] = du.y * tau * iL; o[5] = du.z * tau * iL;
        float qj[9];
        R.dirs(j, qj);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                o[6 + 3 * a + b] = qj[3 * a] * qc[3 * b] + qj[3 * a + 1] * qc[3 * b + 1] + qj[3 * a + 2] * qc[3 * b + 2];
        const V3 wj = R.omega(j);
        o[12] = wj.x * tau; o[13] = wj.y * tau; o[14] = wj.z * tau;
        o[15] = 1.f;
    }
    emit16(o, 16 * (D + 2), g, raw, xn, mu, isd);
}

__device__ inline void window_features(const WinArgs &A, int64_t g, float *raw, __bf16 *xn, const float *mu,
                                const float *isd)
{
    const int r = A.win_rod[g];
    const Rod R(A.B, r);
    const int n = R.n;
    const int w = (int)(g - A.win_first[r]);
    const int c = w < n ? w : n - 1;
    const int p = w < n ? w : n;
    const float *rf = A.rodf + (int64_t)r * NRF;
    float qc[9];
    R.dirs(c, qc);
    const float L = R.lh(c);
    const float iL = 1.f / L;
    const float tau = A.tau;
    const V3 uc = 0.5f * (R.node_v(c) + R.node_v(c + 1));
    emit_slot<-2>(R, c, n, qc, uc, iL, tau, g, raw, xn, mu, isd);
    emit_slot<-1>(R, c, n, qc, uc, iL, tau, g, raw, xn, mu, isd);
    emit_slot<0>(R, c, n, qc, uc, iL, tau, g, raw, xn, mu, isd);
    emit_slot<1>(R, c, n, qc, uc, iL, tau, g, raw, xn, mu, isd);
    emit_slot<2>(R, c, n, qc, uc, iL, tau, g, raw, xn, mu, isd);
    float gl[16];
    const V3 vp = matvec(qc, R.node_v(p));
    gl[0] = vp.x * tau * iL; gl[1] = vp.y * tau * iL; gl[2] = vp.z * tau * iL;
    const V3 ec = R.edge(c);
    const V3 rp = matvec(qc, (p == c ? -0.5f : 0.5f) * ec);
    gl[3] = rp.x * iL; gl[4] = rp.y * iL; gl[5] = rp.z * iL;
    gl[6] = rf[RF_LOGE];
    gl[7] = rf[RF_RADIUS] * iL;
    gl[8] = log10f(tau / (L * L * rf[RF_SQRT_RHOA_EI]));
    gl[9] = rf[RF_ALPHA];
    gl[10] = rf[RF_CLAMP0];
    gl[11] = (float)c / (float)n;
    gl[12] = w == n ? 1.f : 0.f;
    gl[13] = rf[RF_AMP];
    const float2 sc = A.phase[r];
    gl[14] = sc.x;
    gl[15] = sc.y;
    emit16(gl, 80, g, raw, xn, mu, isd);
}

// One wave per workgroup.  BF16 rows are staged in LDS (64 rows x 192 bytes)
// and written out as lane-contiguous 16-byte chunks, so every store
// instruction covers 1 KB of consecutive memory.
constexpr int FEAT_BLOCK = 64;
constexpr int ROW_BF16 = N_FEAT;   // 192 bytes

__global__ __launch_bounds__(FEAT_BLOCK) void features_kernel(const WinArgs A, float *raw, __bf16 *xn, const float *mu,
                                                             const float *isd)
{
    __shared__ __attribute__((aligned(16))) __bf16 rows[FEAT_BLOCK * ROW_BF16];
    const int64_t g0 = (int64_t)blockIdx.x * FEAT_BLOCK;
    const int64_t g = g0 + threadIdx.x;
    if (g < A.n_windows) window_features(A, g, raw, xn ? rows + threadIdx.x * ROW_BF16 : nullptr, mu, isd);
    if (!xn) return;
    __syncthreads();
    const int64_t nrows = A.n_windows - g0 < FEAT_BLOCK ? A.n_windows - g0 : FEAT_BLOCK;
    const int chunks = (int)nrows * (ROW_BF16 * 2 / 16);
    const uint4 *src = reinterpret_cast<const uint4 *>(rows);
    uint4 *dst = reinterpret_cast<uint4 *>(xn + g0 * N_FEAT);
    for (int k = threadIdx.x; k < chunks; k += FEAT_BLOCK) dst[k] = src[k];
}


// ---------------------------------------------------------------- targets
// S0 is the state at t, A.B the state at t + tau (same layout)
__global__ void targets_kernel(const WinArgs A, const DevBatch<float> S0, float *tgt, float *mask)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= A.n_windows) return;
    const int r = A.win_rod[g];
    const Rod R1(A.B, r), R0(S0, r);
    const int n = R1.n;
    const int w = (int)(g - A.win_first[r]);
    const int c = w < n ? w : n - 1;
    const int p = w < n ? w : n;
    float q0[9], q1[9];
    R0.dirs(c, q0);
    R1.dirs(c, q1);
    const float iL = 1.f / R0.lh(c);
    // node p displacement: anchor plus the edges before p
    V3 dr = R1.anchor() - R0.anchor();
    for (int m = 0; m < p; ++m) dr = dr + (R1.edge(m) - R0.edge(m));
    const V3 v0 = R0.node_v(p);
    const V3 a = matvec(q0, dr - A.tau * v0);
    const V3 b = matvec(q0, R1.node_v(p) - v0);
    float *t = tgt + g * N_OUT;
    float *mk = mask + g * N_OUT;
    t[0] = a.x * iL; t[1] = a.y * iL; t[2] = a.z * iL;
    t[3] = b.x * A.tau * iL; t[4] = b.y * A.tau * iL; t[5] = b.z * A.tau * iL;
    for (int k = 0; k < 6; ++k) mk[k] = 1.f;
    if (w < n) {
        const V3 w0 = R0.omega(c);
        const V3 th = log_rel(q0, q1) - A.tau * w0;
        const V3 dw = R1.omega(c) - w0;
        t[6] = th.x; t[7] = th.y; t[8] = th.z;
        t[9] = dw.x * A.tau; t[10] = dw.y * A.tau; t[11] = dw.z * A.tau;
        for (int k = 6; k < 12; ++k) mk[k] = 1.f;
    } else {
        for (int k = 6; k < 12; ++k) { t[k] = 0.f; mk[k] = 0.f; }
    }
}

// ---------------------------------------------------------------- apply
// deltas y [window][ldy]: raw = y * sd + mu (sd = NULL: y is raw already).
// Phase 1 (one thread per window): lab displacement of the target node into
// disp [window][3], node velocity update.  Skips rods with skip[r] != 0.
// One Newton-Schulz step towards the orthogonal polar factor, Q <- Q (3I - Q^T Q) / 2:
// an orthonormality error e becomes O(e^2), so FP32 round-off drift carried in
// by the plain step (about 1e-8 per step) is removed at every coarse step.
__device__ inline void polar_step(float q[9])
{
    float g[9];   // Q^T Q
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) g[3 * a + b] = q[a] * q[b] + q[3 + a] * q[3 + b] + q[6 + a] * q[6 + b];
    float o[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            float acc = 0.f;
            for (int c = 0; c < 3; ++c) acc += q[3 * a + c] * ((c == b ? 3.f : 0.f) - g[3 * c + b]);
            o[3 * a + b] = 0.5f * acc;
        }
    for (int k = 0; k < 9; ++k) q[k] = o[k];
}

__global__ void apply_nodes_kernel(const WinArgs A, const float *y, int ldy, const float *mu, const float *sd,
                                   const int32_t *skip, float *disp)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= A.n_windows) return;
    const int r = A.win_rod[g];
    const Rod R(A.B, r);
    const int n = R.n;
    const int w = (int)(g - A.win_first[r]);
    const int c = w < n ? w : n - 1;
    const int p = w < n ? w : n;
    float d[6];
    for (int k = 0; k < 6; ++k) d[k] = sd ? y[g * ldy + k] * sd[k] + mu[k] : y[g * ldy + k];
    const int flags = A.B.rod_flags[r];
    const bool fixed = (p == 0 && (flags & rodk::FLAG_CLAMP0)) || (p == n && (flags & rodk::FLAG_CLAMP1));
    if ((skip && skip[r]) || fixed) {
        disp[g * 3] = disp[g * 3 + 1] = disp[g * 3 + 2] = 0.f;
        return;
    }
    float qc[9];
    R.dirs(c, qc);
    const float L = R.lh(c);
    const V3 dr = L * matTvec(qc, V3{d[0], d[1], d[2]}) + A.tau * R.node_v(p);   // free flight + learned part
    const V3 dv = matTvec(qc, V3{d[3], d[4], d[5]});
    disp[g * 3] = dr.x;
    disp[g * 3 + 1] = dr.y;
    disp[g * 3 + 2] = dr.z;
    const float s = L / A.tau;
    float *st = A.B.state;
    const int64_t NS = A.B.n_slots;
    float *v0, *v1, *v2;
    if (p < n) {
        v0 = &st[rodk::VX * NS + R.s0 + p]; v1 = &st[rodk::VY * NS + R.s0 + p]; v2 = &st[rodk::VZ * NS + R.s0 + p];
    } else {
        v0 = &A.B.tail[rodk::TVX * A.B.n_rods + r]; v1 = &A.B.tail[rodk::TVY * A.B.n_rods + r];
        v2 = &A.B.tail[rodk::TVZ * A.B.n_rods + r];
    }
    *v0 += dv.x * s;
    *v1 += dv.y * s;
    *v2 += dv.z * s;
    // displacements and velocities; the edges are checked by phase 2
    if (!(isfinite(*v0) && isfinite(*v1) && isfinite(*v2) && isfinite(dr.x) && isfinite(dr.y) && isfinite(dr.z)))
        atomicOr(&A.B.nonfinite[r], ROD_FLAG_NONFINITE);
}

// Phase 2 (one thread per element): edge, anchor, director and omega.
__global__ void apply_elems_kernel(const WinArgs A, const float *y, int ldy, const float *mu, const float *sd,
                                   const int32_t *skip, const float *disp, const int32_t *elem_rod,
                                   const int64_t *elem_first, int64_t n_elems)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    const int r = elem_rod[e];
    if (skip && skip[r]) return;
    const Rod R(A.B, r);
    const int n = R.n;
    const int c = (int)(e - elem_first[r]);
    const int64_t g = A.win_first[r] + c;        // window c targets node c / element c
    float *st = A.B.state;
    const int64_t NS = A.B.n_slots;
    const int64_t sl = R.s0 + c;
    st[rodk::RX * NS + sl] += disp[(g + 1) * 3] - disp[g * 3];
    st[rodk::RY * NS + sl] += disp[(g + 1) * 3 + 1] - disp[g * 3 + 1];
    st[rodk::RZ * NS + sl] += disp[(g + 1) * 3 + 2] - disp[g * 3 + 2];
    if (c == 0) {
        A.B.tail[rodk::TRX * A.B.n_rods + r] += disp[g * 3];
        A.B.tail[rodk::TRY * A.B.n_rods + r] += disp[g * 3 + 1];
        A.B.tail[rodk::TRZ * A.B.n_rods + r] += disp[g * 3 + 2];
    }
    bool ok = isfinite(st[rodk::RX * NS + sl]) && isfinite(st[rodk::RY * NS + sl]) && isfinite(st[rodk::RZ * NS + sl]);
    const int flags = A.B.rod_flags[r];
    const bool fixed = (c == 0 && (flags & rodk::FLAG_CLAMP0)) || (c == n - 1 && (flags & rodk::FLAG_CLAMP1));
    if (!fixed) {
        float d[6];
        for (int k = 0; k < 6; ++k) d[k] = sd ? y[g * ldy + 6 + k] * sd[6 + k] + mu[6 + k] : y[g * ldy + 6 + k];
        float q[9];
        R.dirs(c, q);
        const V3 w0 = R.omega(c);
        rotate_left(q, V3{-(d[0] + w0.x * A.tau), -(d[1] + w0.y * A.tau), -(d[2] + w0.z * A.tau)});
        polar_step(q);
        for (int k = 0; k < 9; ++k) {
            st[(rodk::Q00 + k) * NS + sl] = q[k];
            ok = ok && isfinite(q[k]);
        }
        const float it = 1.f / A.tau;
        st[rodk::WX * NS + sl] += d[3] * it;
        st[rodk::WY * NS + sl] += d[4] * it;
        st[rodk::WZ * NS + sl] += d[5] * it;
        ok = ok && isfinite(st[rodk::WX * NS + sl]) && isfinite(st[rodk::WY * NS + sl]) && isfinite(st[rodk::WZ * NS + sl]);
    }
    if (!ok) atomicOr(&A.B.nonfinite[r], ROD_FLAG_NONFINITE);
}

// ---------------------------------------------------------------- training rows
// Minibatch rows idx[i] of the raw tables, standardised: 16 threads per row,
// thread c < 12 moves features 8c..8c+7 (two 16-byte loads, one 16-byte store
// of eight BF16 values), threads 12-14 four targets and four mask entries each.
__global__ void gather_rows_kernel(const float *fraw, const float *traw, const float *mraw, const int64_t *idx,
                                   int64_t rows, const float *mu_x, const float *isd_x, const float *mu_t,
                                   const float *sd_t, __bf16 *x, float *t, float *m)
{
    typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = g >> 4;
    const int c = (int)(g & 15);
    if (i >= rows || c == 15) return;
    const int64_t s = idx[i];
    if (c < 12) {
        const float4 *src = reinterpret_cast<const float4 *>(fraw + s * N_FEAT + 8 * c);
        const float4 a = src[0], b = src[1];
        const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        bf16x8_t o;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * c + j;
            o[j] = (__bf16)((f[j] - mu_x[k]) * isd_x[k]);
        }
        *reinterpret_cast<bf16x8_t *>(x + i * N_FEAT + 8 * c) = o;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * (c - 12) + j;
            t[i * N_OUT + k] = (traw[s * N_OUT + k] - mu_t[k]) / sd_t[k];
            m[i * N_OUT + k] = mraw[s * N_OUT + k];
        }
    }
}

// Column statistics of a row-major [rows][cols] table over the entries whose
// mask (same shape, or NULL) is nonzero: out[3 * j] = count, sum, sum of squares.
__global__ void colstats_kernel(const float *a, const float *mask, int64_t rows, int cols, double *out)
{
    __shared__ double red[3][256];
    const int j = blockIdx.x;
    double c = 0, s = 0, q = 0;
    for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
        const float m = mask ? mask[i * cols + j] : 1.f;
        if (m != 0.f) {
            const double v = a[i * cols + j];
            c += 1;
            s += v;
            q += v * v;
        }
    }
    red[0][threadIdx.x] = c;
    red[1][threadIdx.x] = s;
    red[2][threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) out[3 * j + k] = red[k][0];
}

// ---------------------------------------------------------------- judge
// The apply step in one pass: one workgroup per rod, one thread per element
// (the last one also takes window n).  Every thread reads what it needs of the
// pre-step state and the outputs, publishes its node displacement in LDS, and
// after one barrier writes its edge, velocity, frame and angular velocity:
// the same arithmetic as apply_nodes_kernel and apply_elems_kernel.
constexpr int APPLY_MAX_THREADS = 512;

__global__ __launch_bounds__(APPLY_MAX_THREADS) void apply_rod_kernel(const WinArgs A, const float *y, int ldy,
                                                                      const float *mu, const float *sd,
                                                                      const int32_t *skip)
{
    __shared__ V3 sdisp[APPLY_MAX_THREADS + 1];
    const int r = blockIdx.x;
    if (skip && skip[r]) return;   // uniform over the workgroup
    const Rod R(A.B, r);
    const int n = R.n;
    const int c = threadIdx.x;
    const bool on = c < n;
    const int flags = A.B.rod_flags[r];
    const int64_t g = A.win_first[r] + c;
    auto out = [&](int64_t row, int k) { return sd ? y[row * ldy + k] * sd[k] + mu[k] : y[row * ldy + k]; };
    float qc[9];
    float L = 0.f;
    V3 dv{0.f, 0.f, 0.f}, dvn{0.f, 0.f, 0.f};
    if (on) {
        R.dirs(c, qc);
        L = R.lh(c);
        const bool fixed = (c == 0 && (flags & rodk::FLAG_CLAMP0));
        V3 dr{0.f, 0.f, 0.f};
        if (!fixed) {
            dr = L * matTvec(qc, V3{out(g, 0), out(g, 1), out(g, 2)}) + A.tau * R.node_v(c);
            dv = (L / A.tau) * matTvec(qc, V3{out(g, 3), out(g, 4), out(g, 5)});
        }
        sdisp[c] = dr;
        if (c == n - 1) {   // window n: node n, centred on element n - 1
            V3 drn{0.f, 0.f, 0.f};
            if (!(flags & rodk::FLAG_CLAMP1)) {
                drn = L * matTvec(qc, V3{out(g + 1, 0), out(g + 1, 1), out(g + 1, 2)}) + A.tau * R.node_v(n);
                dvn = (L / A.tau) * matTvec(qc, V3{out(g + 1, 3), out(g + 1, 4), out(g + 1, 5)});
            }
            sdisp[n] = drn;
        }
    }
    __syncthreads();
    if (!on) return;
    float *st = A.B.state;
    const int64_t NS = A.B.n_slots;
    const int64_t sl = R.s0 + c;
    const V3 d0 = sdisp[c], d1 = sdisp[c + 1];
    bool ok = true;   // every value this thread writes is finite
    auto add = [&](float *a, float dlt) {
        const float v = *a + dlt;
        *a = v;
        ok = ok && isfinite(v);
    };
    add(&st[rodk::RX * NS + sl], d1.x - d0.x);
    add(&st[rodk::RY * NS + sl], d1.y - d0.y);
    add(&st[rodk::RZ * NS + sl], d1.z - d0.z);
    if (c == 0) {
        add(&A.B.tail[rodk::TRX * A.B.n_rods + r], d0.x);
        add(&A.B.tail[rodk::TRY * A.B.n_rods + r], d0.y);
        add(&A.B.tail[rodk::TRZ * A.B.n_rods + r], d0.z);
    }
    add(&st[rodk::VX * NS + sl], dv.x);
    add(&st[rodk::VY * NS + sl], dv.y);
    add(&st[rodk::VZ * NS + sl], dv.z);
    if (c == n - 1) {
        add(&A.B.tail[rodk::TVX * A.B.n_rods + r], dvn.x);
        add(&A.B.tail[rodk::TVY * A.B.n_rods + r], dvn.y);
        add(&A.B.tail[rodk::TVZ * A.B.n_rods + r], dvn.z);
    }
    const bool fixed_e = (c == 0 && (flags & rodk::FLAG_CLAMP0)) || (c == n - 1 && (flags & rodk::FLAG_CLAMP1));
    if (!fixed_e) {
        float d[6];
        for (int k = 0; k < 6; ++k) d[k] = out(g, 6 + k);
        const V3 w0 = R.omega(c);
        rotate_left(qc, V3{-(d[0] + w0.x * A.tau), -(d[1] + w0.y * A.tau), -(d[2] + w0.z * A.tau)});
        polar_step(qc);
        for (int k = 0; k < 9; ++k) {
            st[(rodk::Q00 + k) * NS + sl] = qc[k];
            ok = ok && isfinite(qc[k]);
        }
        const float it = 1.f / A.tau;
        add(&st[rodk::WX * NS + sl], d[3] * it);
        add(&st[rodk::WY * NS + sl], d[4] * it);
        add(&st[rodk::WZ * NS + sl], d[5] * it);
    }
    // a rod the learned step drives to NaN/Inf is flagged like one the plain step does
    if (!ok) atomicOr(&A.B.nonfinite[r], ROD_FLAG_NONFINITE);
}

// Copy rods between two FP32 batches of equal per-rod layout: dst rod k <- src rod map[k]
// (state, constants, tail, per-rod tables).  One thread per (k, element).
__global__ void copy_rods_kernel(DevBatch<float> dst, DevBatch<float> src, const int32_t *map, const int32_t *sel,
                                 int n_map, int n, bool state_only, bool to_src)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_map * n) return;
    const int k = (int)(t / n), i = (int)(t % n);
    if (sel && !sel[k]) return;
    const int rs = map[k];
    // to_src: write the dst batch's rod k back into src rod map[k]
    const DevBatch<float> &from = to_src ? dst : src;
    const DevBatch<float> &to = to_src ? src : dst;
    const int rf = to_src ? k : rs, rt = to_src ? rs : k;
    const int64_t sf = from.rod_slot[rf] + i, stt = to.rod_slot[rt] + i;
    for (int f = 0; f < rodk::N_STATE; ++f) to.state[(int64_t)f * to.n_slots + stt] = from.state[(int64_t)f * from.n_slots + sf];
    if (!state_only)
        for (int f = 0; f < rodk::N_PARAM; ++f)
            to.param[(int64_t)f * to.n_slots + stt] = from.param[(int64_t)f * from.n_slots + sf];
    if (i == 0) {
        for (int f = 0; f < rodk::N_TAIL; ++f) to.tail[(int64_t)f * to.n_rods + rt] = from.tail[(int64_t)f * from.n_rods + rf];
        if (!state_only) {
            for (int f = 0; f < rodk::N_RODP; ++f)
                to.rodp[(int64_t)f * to.n_rods + rt] = from.rodp[(int64_t)f * from.n_rods + rf];
            to.rod_freq[rt] = from.rod_freq[rf];
            to.rod_phase[rt] = from.rod_phase[rf];
            to.rod_flags[rt] = from.rod_flags[rf];
        }
        to.nonfinite[rt] = from.nonfinite[rf];   // the flags travel with the state they describe
    }
}

// Per judged rod k: max_j |r_j - r_j(ref)| / L (L = sum of rest lengths) of
// the main batch's rod map[k] against the judge batch's rod k, and the main
// batch's director orthonormality error max |Q Q^T - I|.
__global__ void judge_errors_kernel(DevBatch<float> main, DevBatch<float> ref, const int32_t *map, int n_map,
                                    float *err)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_map) return;
    const Rod Rm(main, map[k]), Rr(ref, k);
    const int n = Rm.n;
    V3 d = Rm.anchor() - Rr.anchor();
    float L = 0.f, worst = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z), orth = 0.f;
    for (int i = 0; i < n; ++i) {
        L += Rm.lh(i);
        d = d + (Rm.edge(i) - Rr.edge(i));
        worst = fmaxf(worst, sqrtf(d.x * d.x + d.y * d.y + d.z * d.z));
        float q[9];
        Rm.dirs(i, q);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const float s = q[3 * a] * q[3 * b] + q[3 * a + 1] * q[3 * b + 1] + q[3 * a + 2] * q[3 * b + 2];
                orth = fmaxf(orth, fabsf(s - (a == b ? 1.f : 0.f)));
            }
    }
    err[2 * k] = worst / L;
    err[2 * k + 1] = orth;
}

// Counter-based normal deviates: the splitmix64 output function (Steele, Lea
// and Flood 2014) hashes (seed, key) to 64 bits, Box-Muller turns two 24-bit
// uniforms into one N(0, 1) value.
__device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ inline float gauss(uint64_t seed, uint64_t key)
{
    const uint64_t h = mix64(seed ^ mix64(key));
    const float u1 = ((float)(h >> 40) + 0.5f) * (1.0f / 16777216.0f);
    const float u2 = ((float)(h & 0xFFFFFFull) + 0.5f) * (1.0f / 16777216.0f);
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}
// key of component a (0-2) of quantity kind (0 position, 1 velocity, 2 rotation, 3 omega) at node/element j of rod r
__device__ inline uint64_t noise_key(int r, int j, int kind, int a)
{
    return ((uint64_t)(uint32_t)r << 32) | ((uint64_t)(uint32_t)j << 4) | (uint64_t)(3 * kind + a);
}

// Perturb the free part of every rod in place: node positions by
// noise[0] lh N(0, 1), node velocities by noise[1] lh / tau N(0, 1), each
// director frame by the rotation exp(-[noise[2] g]x), g ~ N(0, I), and
// angular velocities by noise[3] / tau N(0, 1) (lh of the node's own element,
// element n-1 for node n).  Clamped nodes and elements are left alone.  One
// thread per element: element c moves edge c by the noise of nodes c and c+1.
__global__ void perturb_kernel(DevBatch<float> B, const int32_t *elem_rod, const int64_t *elem_first, int64_t n_elems,
                               float4 noise, float tau, uint64_t seed)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_elems) return;
    const int r = elem_rod[e];
    const Rod R(B, r);
    const int n = R.n;
    const int c = (int)(e - elem_first[r]);
    const int flags = B.rod_flags[r];
    const bool c0 = flags & rodk::FLAG_CLAMP0, c1 = flags & rodk::FLAG_CLAMP1;
    auto node_fixed = [&](int j) { return (j == 0 && c0) || (j == n && c1); };
    auto node_noise = [&](int j, int kind, float scale) -> V3 {
        if (node_fixed(j) || scale == 0.f) return {0.f, 0.f, 0.f};
        const float L = R.lh(j < n ? j : n - 1) * scale;
        return {L * gauss(seed, noise_key(r, j, kind, 0)), L * gauss(seed, noise_key(r, j, kind, 1)),
                L * gauss(seed, noise_key(r, j, kind, 2))};
    };
    float *st = B.state;
    const int64_t NS = B.n_slots, sl = R.s0 + c;
    const V3 d0 = node_noise(c, 0, noise.x), d1 = node_noise(c + 1, 0, noise.x);
    st[rodk::RX * NS + sl] += d1.x - d0.x;
    st[rodk::RY * NS + sl] += d1.y - d0.y;
    st[rodk::RZ * NS + sl] += d1.z - d0.z;
    if (c == 0) {
        B.tail[rodk::TRX * B.n_rods + r] += d0.x;
        B.tail[rodk::TRY * B.n_rods + r] += d0.y;
        B.tail[rodk::TRZ * B.n_rods + r] += d0.z;
    }
    const float vs = noise.y / tau;
    const V3 dv = node_noise(c, 1, vs);
    st[rodk::VX * NS + sl] += dv.x;
    st[rodk::VY * NS + sl] += dv.y;
    st[rodk::VZ * NS + sl] += dv.z;
    if (c == n - 1) {
        const V3 dn = node_noise(n, 1, vs);
        B.tail[rodk::TVX * B.n_rods + r] += dn.x;
        B.tail[rodk::TVY * B.n_rods + r] += dn.y;
        B.tail[rodk::TVZ * B.n_rods + r] += dn.z;
    }
    if ((c == 0 && c0) || (c == n - 1 && c1)) return;
    if (noise.z != 0.f) {
        float q[9];
        R.dirs(c, q);
        const V3 g{gauss(seed, noise_key(r, c, 2, 0)), gauss(seed, noise_key(r, c, 2, 1)),
                   gauss(seed, noise_key(r, c, 2, 2))};
        rotate_left(q, V3{-noise.z * g.x, -noise.z * g.y, -noise.z * g.z});
        for (int k = 0; k < 9; ++k) st[(rodk::Q00 + k) * NS + sl] = q[k];
    }
    const float ws = noise.w / tau;
    st[rodk::WX * NS + sl] += ws * gauss(seed, noise_key(r, c, 3, 0));
    st[rodk::WY * NS + sl] += ws * gauss(seed, noise_key(r, c, 3, 1));
    st[rodk::WZ * NS + sl] += ws * gauss(seed, noise_key(r, c, 3, 2));
}

// ---------------------------------------------------------------- launchers
static inline dim3 blocks(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

hipError_t features(const WinArgs &A, float *raw, __bf16 *xn, const float *mu, const float *isd, hipStream_t s)
{
    hipLaunchKernelGGL(phase_kernel, blocks(A.B.n_rods), dim3(256), 0, s, A.rodf, A.B.n_rods, A.time, A.phase);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    hipLaunchKernelGGL(features_kernel, blocks(A.n_windows, FEAT_BLOCK), dim3(FEAT_BLOCK), 0, s, A, raw, xn, mu, isd);
    return hipGetLastError();
}

hipError_t targets(const WinArgs &A, const DevBatch<float> &S0, float *tgt, float *mask, hipStream_t s)
{
    hipLaunchKernelGGL(targets_kernel, blocks(A.n_windows, 128), dim3(128), 0, s, A, S0, tgt, mask);
    return hipGetLastError();
}

hipError_t apply(const WinArgs &A, const float *y, int ldy, const float *mu, const float *sd, const int32_t *skip,
                 float *disp, const int32_t *elem_rod, const int64_t *elem_first, int64_t n_elems, hipStream_t s,
                 int n_max)
{
    if (n_max > 0 && n_max <= APPLY_MAX_THREADS) {
        const int threads = (n_max + 63) / 64 * 64;
        hipLaunchKernelGGL(apply_rod_kernel, dim3(A.B.n_rods), dim3(threads), 0, s, A, y, ldy, mu, sd, skip);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(apply_nodes_kernel, blocks(A.n_windows), dim3(256), 0, s, A, y, ldy, mu, sd, skip, disp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(apply_elems_kernel, blocks(n_elems), dim3(256), 0, s, A, y, ldy, mu, sd, skip, disp, elem_rod,
                       elem_first, n_elems);
    return hipGetLastError();
}

hipError_t gather_rows(const float *fraw, const float *traw, const float *mraw, const int64_t *idx, int64_t rows,
                       const float *mu_x, const float *isd_x, const float *mu_t, const float *sd_t, __bf16 *x, float *t,
                       float *m, hipStream_t s)
{
    hipLaunchKernelGGL(gather_rows_kernel, blocks(16 * rows), dim3(256), 0, s, fraw, traw, mraw, idx, rows, mu_x, isd_x,
                       mu_t, sd_t, x, t, m);
    return hipGetLastError();
}

hipError_t copy_rods(const DevBatch<float> &dst, const DevBatch<float> &src, const int32_t *map, const int32_t *sel,
                     int n_map, int n, bool state_only, bool to_src, hipStream_t s)
{
    hipLaunchKernelGGL(copy_rods_kernel, blocks((int64_t)n_map * n), dim3(256), 0, s, dst, src, map, sel, n_map, n,
                       state_only, to_src);
    return hipGetLastError();
}

hipError_t perturb(const DevBatch<float> &B, const int32_t *elem_rod, const int64_t *elem_first, int64_t n_elems,
                   const float noise[4], float tau, uint64_t seed, hipStream_t s)
{
    const float4 nz{noise[0], noise[1], noise[2], noise[3]};
    hipLaunchKernelGGL(perturb_kernel, blocks(n_elems), dim3(256), 0, s, B, elem_rod, elem_first, n_elems, nz, tau,
                       seed);
    return hipGetLastError();
}

hipError_t colstats(const float *a, const float *mask, int64_t rows, int cols, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(colstats_kernel, dim3(cols), dim3(256), 0, s, a, mask, rows, cols, out);
    return hipGetLastError();
}

hipError_t judge_errors(const DevBatch<float> &main, const DevBatch<float> &ref, const int32_t *map, int n_map,
                        float *err, hipStream_t s)
{
    hipLaunchKernelGGL(judge_errors_kernel, blocks(n_map, 64), dim3(64), 0, s, main, ref, map, n_map, err);
    return hipGetLastError();
}

}  // namespace surk
