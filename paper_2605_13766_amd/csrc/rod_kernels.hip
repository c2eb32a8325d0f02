// rod_kernels.hip -- gfx950 kernels of the discrete Cosserat-rod step.
//
// Mapping: one lane per element.  A workgroup of 64*W lanes owns a tile of
// whole rods laid out on consecutive lanes; lane i of a rod holds node i
// (v, and r in FP64) and element i (Q, omega, and the edge r_{i+1} - r_i in
// FP32); the rod's last lane also holds node n.
// Each launch loads its tiles' state once, runs `n_sub` position-Verlet
// substeps with the state in registers, and stores it once.  The two-point
// stencils of the difference and averaging operators read the neighbour
// lane's values through LDS (three exchanges per substep, four in FP32).
//
// Model: Elastica++, Methods, "Cosserat rod dynamics", Eq. 1a (linear
// momentum) and Eq. 1b (angular momentum) on the staggered grid of nodes,
// elements and Voronoi points; time stepping per Results,
// "Performance-oriented software design" (position Verlet with the
// kinematic constraints imposed after every stage).
#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>

namespace rodk {

namespace {

template <typename T> struct Coef;
template <> struct Coef<double> {
    static constexpr double rot_series_max = 1e-2;   // theta^2 bound of the series path
    static constexpr double log_series_max = 4e-3;   // |w|^2 bound of the series path
};
template <> struct Coef<float> {
    static constexpr float rot_series_max = 1e-2f;
    static constexpr float log_series_max = 4e-3f;
};

__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float dsqrt(float x) { return sqrtf(x); }
__device__ inline double dsin(double x) { return sin(x); }
__device__ inline float dsin(float x) { return sinf(x); }
__device__ inline double dcos(double x) { return cos(x); }
__device__ inline float dcos(float x) { return cosf(x); }
__device__ inline double datan2(double y, double x) { return atan2(y, x); }
__device__ inline float datan2(float y, float x) { return atan2f(y, x); }

// q <- exp([u]x) q for a row-major director matrix q (rows d1, d2, d3).
// exp([u]x) = I + a [u]x + b [u]x^2 with a = sin(t)/t, b = (1 - cos t)/t^2,
// t = |u|; both are even series in t^2, used for small t.  [u]x acts on the
// columns of q (the lab components of the three directors).
template <typename T>
__device__ inline void rotate_left(T q[9], T ux, T uy, T uz)
{
    const T x = ux * ux + uy * uy + uz * uz;
    T a, b;
    if (x < Coef<T>::rot_series_max) {
        // sin(t)/t = 1 - x/3! + x^2/5! - x^3/7! + x^4/9!
        a = T(1) + x * (T(-1.0 / 6) + x * (T(1.0 / 120) + x * (T(-1.0 / 5040) + x * T(1.0 / 362880))));
        // (1-cos t)/t^2 = 1/2! - x/4! + x^2/6! - x^3/8! + x^4/10!
        b = T(0.5) + x * (T(-1.0 / 24) + x * (T(1.0 / 720) + x * (T(-1.0 / 40320) + x * T(1.0 / 3628800))));
    } else {
        const T t = dsqrt(x);
        a = dsin(t) / t;
        b = (T(1) - dcos(t)) / x;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T c0 = q[j], c1 = q[3 + j], c2 = q[6 + j];
        const T k0 = uy * c2 - uz * c1;
        const T k1 = uz * c0 - ux * c2;
        const T k2 = ux * c1 - uy * c0;
        const T kk0 = uy * k2 - uz * k1;
        const T kk1 = uz * k0 - ux * k2;
        const T kk2 = ux * k1 - uy * k0;
        q[j] = c0 + a * k0 + b * kk0;
        q[3 + j] = c1 + a * k1 + b * kk1;
        q[6 + j] = c2 + a * k2 + b * kk2;
    }
}

// Rotation vector of R = qa qb^T (rows of qa against rows of qb):
// w = ax(R) = sin(t) k, c = (tr R - 1)/2 = cos(t), result = (t / |w|) w.
// t/|w| = asin(s)/s with s = |w| when c > 0, an even series in s^2.
template <typename T>
__device__ inline void log_relative(const T qa[9], const T qb[9], T &u0, T &u1, T &u2)
{
    T R[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            R[3 * a + b] = qa[3 * a] * qb[3 * b] + qa[3 * a + 1] * qb[3 * b + 1] + qa[3 * a + 2] * qb[3 * b + 2];
    const T w0 = T(0.5) * (R[7] - R[5]);
    const T w1 = T(0.5) * (R[2] - R[6]);
    const T w2 = T(0.5) * (R[3] - R[1]);
    const T c = T(0.5) * (R[0] + R[4] + R[8] - T(1));
    const T s2 = w0 * w0 + w1 * w1 + w2 * w2;
    T f;
    if (c > T(0) && s2 < Coef<T>::log_series_max) {
        // asin(s)/s = sum_k (2k)! / (4^k (k!)^2 (2k+1)) s^(2k)
        f = T(1) + s2 * (T(1.0 / 6) + s2 * (T(3.0 / 40) + s2 * (T(5.0 / 112) + s2 * (T(35.0 / 1152)
              + s2 * (T(63.0 / 2816) + s2 * (T(231.0 / 13312) + s2 * T(143.0 / 10240)))))));
    } else {
        const T s = dsqrt(s2);
        f = datan2(s, c) / s;
    }
    u0 = f * w0;
    u1 = f * w1;
    u2 = f * w2;
}

template <typename T>
__device__ inline bool finite3(T a, T b, T c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

}  // namespace

// One launch: n_sub position-Verlet substeps for every tile (grid-stride).
//
// FP64 keeps node positions.  FP32 keeps, per element, the edge vector
// e_i = r_{i+1} - r_i and, per rod, the position of node 0 (the anchor): the
// drift r_j += h/2 v_j becomes e_i += h/2 (v_{i+1} - v_i), anchor += h/2 v_0,
// which is the same update in exact arithmetic but keeps the strains at
// FP32 relative precision (absolute FP32 positions would round each drift
// increment against the rod's whole length).
template <typename T, int W>
__global__ __launch_bounds__(64 * W) void rod_step_kernel(const DevBatch<T> B, int n_sub)
{
    constexpr int TL = 64 * W;
    constexpr bool EDGE = sizeof(T) == 4;
    constexpr int NX1 = EDGE ? 9 : 15;
    __shared__ T xa[NX1][TL + 1];          // from the right: (r, v,) Q
    __shared__ T xb[TL + 1];               // from the right: current length
    __shared__ T xc[9][TL + 1];            // from the left: n, M, y
    __shared__ T xd[EDGE ? 3 : 1][TL + 1]; // from the right: post-kick v (edge form)

    const int lane = threadIdx.x;
    const int64_t NS = B.n_slots;
    const int64_t step0 = *B.step;
    const T h = T(B.dt);
    const T hh = T(0.5 * B.dt);
    const int left = lane > 0 ? lane - 1 : 0;

    for (int tile = blockIdx.x; tile < B.n_tiles; tile += gridDim.x) {
        const int64_t s = (int64_t)tile * TL + lane;
        const int rod = B.slot_rod[s];
        const bool valid = rod >= 0;
        const int rr = valid ? rod : 0;
        const int i = B.slot_idx[s];
        const int n = valid ? B.rod_n[rr] : 1;
        const int flags = valid ? B.rod_flags[rr] : 0;
        const bool last = valid && (i == n - 1);
        const bool hasv = valid && (i < n - 1);
        const bool first = i == 0;
        const bool fix0 = first && (flags & FLAG_CLAMP0);
        const bool fix1 = last && (flags & FLAG_CLAMP1);

        // ---- state: r0..2 is node i's position (FP64) or element i's edge (FP32);
        // t0..2 is node n's position (FP64, last lane) or node 0's (FP32, first lane)
        const T *st = B.state + s;
        T r0 = st[RX * NS], r1 = st[RY * NS], r2 = st[RZ * NS];
        T v0 = st[VX * NS], v1 = st[VY * NS], v2 = st[VZ * NS];
        T q[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k] = st[(Q00 + k) * NS];
        T w0 = st[WX * NS], w1 = st[WY * NS], w2 = st[WZ * NS];
        T t0 = 0, t1 = 0, t2 = 0, u0 = 0, u1 = 0, u2 = 0;   // tail position, node n velocity
        if (EDGE ? (valid && first) : last) {
            t0 = B.tail[TRX * B.n_rods + rr]; t1 = B.tail[TRY * B.n_rods + rr]; t2 = B.tail[TRZ * B.n_rods + rr];
        }
        if (last) {
            u0 = B.tail[TVX * B.n_rods + rr]; u1 = B.tail[TVY * B.n_rods + rr]; u2 = B.tail[TVZ * B.n_rods + rr];
        }
        // ---- constants
        const T *pp = B.param + s;
        const T inv_m = pp[P_INV_M * NS], lh = pp[P_LH * NS], inv_lh = pp[P_INV_LH * NS];
        const T J1 = pp[P_J1 * NS], S1 = pp[P_S1 * NS], S3 = pp[P_S3 * NS];
        const T Dh = pp[P_DH * NS], inv_Dh = pp[P_INV_DH * NS], B1 = pp[P_B1 * NS], B3 = pp[P_B3 * NS];
        const T k00 = pp[P_K0X * NS], k01 = pp[P_K0Y * NS], k02 = pp[P_K0Z * NS];
        const T J3 = T(2) * J1;
        const T inv_J1 = T(1) / J1, inv_J3 = T(1) / J3;
        const T gamma = B.rodp[R_GAMMA * B.n_rods + rr];
        T inv_mt = 0, f0 = 0, f1 = 0, f2 = 0;
        if (last) {
            inv_mt = B.rodp[R_INV_M_TAIL * B.n_rods + rr];
            f0 = B.rodp[R_FX * B.n_rods + rr]; f1 = B.rodp[R_FY * B.n_rods + rr]; f2 = B.rodp[R_FZ * B.n_rods + rr];
        }
        // distributed couple amplitude times rest length; its time factor
        // sin(2 pi f t + phi) at the substep midpoints by rotation recurrence
        T c0 = 0, c1 = 0, c2 = 0;
        double ps = 0.0, pc = 1.0, ds = 0.0, dc = 1.0;
        if (valid && (flags & FLAG_COUPLE)) {
            c0 = B.rodp[R_CX * B.n_rods + rr] * lh;
            c1 = B.rodp[R_CY * B.n_rods + rr] * lh;
            c2 = B.rodp[R_CZ * B.n_rods + rr] * lh;
            const double fr = B.rod_freq[rr];
            const double ph = 2.0 * M_PI * fr * (B.t0 + ((double)step0 + 0.5) * B.dt) + B.rod_phase[rr];
            ps = sin(ph);
            pc = cos(ph);
            const double dp = 2.0 * M_PI * fr * B.dt;
            ds = sin(dp);
            dc = cos(dp);
        }

        // edge form: velocity of node i+1 (refreshed after every kick)
        T vn0 = 0, vn1 = 0, vn2 = 0;
        if constexpr (EDGE) {
            xd[0][lane] = v0; xd[1][lane] = v1; xd[2][lane] = v2;
            __syncthreads();
            if (last) { vn0 = u0; vn1 = u1; vn2 = u2; }
            else { vn0 = xd[0][lane + 1]; vn1 = xd[1][lane + 1]; vn2 = xd[2][lane + 1]; }
        }

        for (int sub = 0; sub < n_sub; ++sub) {
            // ---- half drift (constraints hold: clamped v, omega are zero)
            if constexpr (EDGE) {
                r0 += hh * (vn0 - v0); r1 += hh * (vn1 - v1); r2 += hh * (vn2 - v2);
                t0 += hh * v0; t1 += hh * v1; t2 += hh * v2;
            } else {
                r0 += hh * v0; r1 += hh * v1; r2 += hh * v2;
                t0 += hh * u0; t1 += hh * u1; t2 += hh * u2;
            }
            rotate_left(q, -hh * w0, -hh * w1, -hh * w2);

            // ---- exchange 1: neighbour element (and node)
            if constexpr (!EDGE) {
                xa[9][lane] = r0; xa[10][lane] = r1; xa[11][lane] = r2;
                xa[12][lane] = v0; xa[13][lane] = v1; xa[14][lane] = v2;
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) xa[k][lane] = q[k];
            __syncthreads();
            T d0, d1, d2;
            if constexpr (EDGE) {
                d0 = r0; d1 = r1; d2 = r2;
            } else {
                if (last) {
                    d0 = t0 - r0; d1 = t1 - r1; d2 = t2 - r2;
                    vn0 = u0; vn1 = u1; vn2 = u2;
                } else {
                    d0 = xa[9][lane + 1] - r0; d1 = xa[10][lane + 1] - r1; d2 = xa[11][lane + 1] - r2;
                    vn0 = xa[12][lane + 1]; vn1 = xa[13][lane + 1]; vn2 = xa[14][lane + 1];
                }
            }
            T qn[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) qn[k] = xa[k][lane + 1];

            // ---- kinematics and shear/stretch strain of element i
            const T l2 = d0 * d0 + d1 * d1 + d2 * d2;
            const T l = dsqrt(l2);
            const T inv_l = T(1) / l;
            const T e = l * inv_lh;
            const T inv_e = lh * inv_l;
            const T edot = ((d0 * (vn0 - v0) + d1 * (vn1 - v1) + d2 * (vn2 - v2)) * inv_l) * inv_lh;
            // sigma = Q dr / lh - e3
            const T sg0 = (q[0] * d0 + q[1] * d1 + q[2] * d2) * inv_lh;
            const T sg1 = (q[3] * d0 + q[4] * d1 + q[5] * d2) * inv_lh;
            const T sg2 = (q[6] * d0 + q[7] * d1 + q[8] * d2) * inv_lh - T(1);
            const T ss0 = S1 * sg0, ss1 = S1 * sg1, ss2 = S3 * sg2;
            // internal force n = Q^T S sigma / e (lab)
            const T nf0 = (q[0] * ss0 + q[3] * ss1 + q[6] * ss2) * inv_e;
            const T nf1 = (q[1] * ss0 + q[4] * ss1 + q[7] * ss2) * inv_e;
            const T nf2 = (q[2] * ss0 + q[5] * ss1 + q[8] * ss2) * inv_e;

            // ---- exchange 2: neighbour length
            xb[lane] = l;
            __syncthreads();
            const T ln = xb[lane + 1];

            // ---- curvature, bending/twisting moment at Voronoi point i
            T M0 = 0, M1 = 0, M2 = 0, y0 = 0, y1 = 0, y2 = 0;
            if (hasv) {
                T k0, k1, k2;
                log_relative(q, qn, k0, k1, k2);
                k0 *= inv_Dh; k1 *= inv_Dh; k2 *= inv_Dh;
                const T eps = (l + ln) * (T(0.5) * inv_Dh);
                const T ie3 = T(1) / (eps * eps * eps);
                M0 = B1 * (k0 - k00) * ie3;
                M1 = B1 * (k1 - k01) * ie3;
                M2 = B3 * (k2 - k02) * ie3;
                y0 = (k1 * M2 - k2 * M1) * Dh;
                y1 = (k2 * M0 - k0 * M2) * Dh;
                y2 = (k0 * M1 - k1 * M0) * Dh;
            }

            // ---- exchange 3: left neighbour's force and moments
            xc[0][lane] = nf0; xc[1][lane] = nf1; xc[2][lane] = nf2;
            xc[3][lane] = M0; xc[4][lane] = M1; xc[5][lane] = M2;
            xc[6][lane] = y0; xc[7][lane] = y1; xc[8][lane] = y2;
            __syncthreads();
            T np0 = 0, np1 = 0, np2 = 0, Mp0 = 0, Mp1 = 0, Mp2 = 0, yp0 = 0, yp1 = 0, yp2 = 0;
            if (!first) {
                np0 = xc[0][left]; np1 = xc[1][left]; np2 = xc[2][left];
                Mp0 = xc[3][left]; Mp1 = xc[4][left]; Mp2 = xc[5][left];
                yp0 = xc[6][left]; yp1 = xc[7][left]; yp2 = xc[8][left];
            }

            // ---- Eq. 1a at node i (and node n on the last lane)
            const T a0 = (nf0 - np0) * inv_m - gamma * v0;
            const T a1 = (nf1 - np1) * inv_m - gamma * v1;
            const T a2 = (nf2 - np2) * inv_m - gamma * v2;

            // ---- Eq. 1b at element i
            // Q t = (sigma + e3) / e
            const T qt0 = sg0 * inv_e, qt1 = sg1 * inv_e, qt2 = (sg2 + T(1)) * inv_e;
            const T jw0 = J1 * w0 * inv_e, jw1 = J1 * w1 * inv_e, jw2 = J3 * w2 * inv_e;
            const T ede = edot * inv_e;
            const T tq0 = (M0 - Mp0) + T(0.5) * (yp0 + y0) + (qt1 * ss2 - qt2 * ss1) * lh
                        + (jw1 * w2 - jw2 * w1) + jw0 * ede + c0 * T(ps);
            const T tq1 = (M1 - Mp1) + T(0.5) * (yp1 + y1) + (qt2 * ss0 - qt0 * ss2) * lh
                        + (jw2 * w0 - jw0 * w2) + jw1 * ede + c1 * T(ps);
            const T tq2 = (M2 - Mp2) + T(0.5) * (yp2 + y2) + (qt0 * ss1 - qt1 * ss0) * lh
                        + (jw0 * w1 - jw1 * w0) + jw2 * ede + c2 * T(ps);
            const T al0 = e * inv_J1 * tq0 - gamma * w0;
            const T al1 = e * inv_J1 * tq1 - gamma * w1;
            const T al2 = e * inv_J3 * tq2 - gamma * w2;

            // ---- kick, then constraints
            v0 += h * a0; v1 += h * a1; v2 += h * a2;
            w0 += h * al0; w1 += h * al1; w2 += h * al2;
            if (last) {
                u0 += h * ((f0 - nf0) * inv_mt - gamma * u0);
                u1 += h * ((f1 - nf1) * inv_mt - gamma * u1);
                u2 += h * ((f2 - nf2) * inv_mt - gamma * u2);
            }
            if (fix0) { v0 = v1 = v2 = 0; w0 = w1 = w2 = 0; }
            if (fix1) { u0 = u1 = u2 = 0; w0 = w1 = w2 = 0; }

            // ---- edge form: exchange 4, the post-kick velocity of node i+1
            if constexpr (EDGE) {
                xd[0][lane] = v0; xd[1][lane] = v1; xd[2][lane] = v2;
                __syncthreads();
                if (last) { vn0 = u0; vn1 = u1; vn2 = u2; }
                else { vn0 = xd[0][lane + 1]; vn1 = xd[1][lane + 1]; vn2 = xd[2][lane + 1]; }
            }

            // ---- second half drift
            if constexpr (EDGE) {
                r0 += hh * (vn0 - v0); r1 += hh * (vn1 - v1); r2 += hh * (vn2 - v2);
                t0 += hh * v0; t1 += hh * v1; t2 += hh * v2;
            } else {
                r0 += hh * v0; r1 += hh * v1; r2 += hh * v2;
                t0 += hh * u0; t1 += hh * u1; t2 += hh * u2;
            }
            rotate_left(q, -hh * w0, -hh * w1, -hh * w2);

            // advance the couple's phase by one step
            const double nps = ps * dc + pc * ds;
            pc = pc * dc - ps * ds;
            ps = nps;
        }

        if (valid) {
            T *so = B.state + s;
            so[RX * NS] = r0; so[RY * NS] = r1; so[RZ * NS] = r2;
            so[VX * NS] = v0; so[VY * NS] = v1; so[VZ * NS] = v2;
#pragma unroll
            for (int k = 0; k < 9; ++k) so[(Q00 + k) * NS] = q[k];
            so[WX * NS] = w0; so[WY * NS] = w1; so[WZ * NS] = w2;
            bool ok = finite3(r0, r1, r2) && finite3(v0, v1, v2) && finite3(w0, w1, w2)
                    && finite3(q[0], q[1], q[2]) && finite3(q[3], q[4], q[5]) && finite3(q[6], q[7], q[8]);
            if (EDGE ? first : last) {
                B.tail[TRX * B.n_rods + rr] = t0; B.tail[TRY * B.n_rods + rr] = t1; B.tail[TRZ * B.n_rods + rr] = t2;
                ok = ok && finite3(t0, t1, t2);
            }
            if (last) {
                B.tail[TVX * B.n_rods + rr] = u0; B.tail[TVY * B.n_rods + rr] = u1; B.tail[TVZ * B.n_rods + rr] = u2;
                ok = ok && finite3(u0, u1, u2);
            }
            if (!ok) B.nonfinite[rr] = 1;
        }
        __syncthreads();   // LDS reuse by the next tile
    }
}

__global__ void advance_kernel(int64_t *step, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += n;
}

// Per-rod energies, one thread per rod walking its slots (off the step path).
// FP32 batches hold edge vectors: node n = anchor + sum of edges (in FP64).
template <typename T>
__global__ void rod_energy_kernel(const DevBatch<T> B, double *out)
{
    constexpr bool EDGE = sizeof(T) == 4;
    const int rod = blockIdx.x * blockDim.x + threadIdx.x;
    if (rod >= B.n_rods) return;
    const int64_t NS = B.n_slots;
    const int n = B.rod_n[rod];
    const int64_t s0 = B.rod_slot[rod];
    auto S = [&](int f, int64_t s) -> double { return (double)B.state[f * NS + s]; };
    auto P = [&](int f, int64_t s) -> double { return (double)B.param[f * NS + s]; };
    auto RP = [&](int f) -> double { return (double)B.rodp[f * B.n_rods + rod]; };
    double Tl = 0, Tr = 0, Us = 0, Ub = 0;
    double tr0 = (double)B.tail[TRX * B.n_rods + rod];
    double tr1 = (double)B.tail[TRY * B.n_rods + rod];
    double tr2 = (double)B.tail[TRZ * B.n_rods + rod];
    const double tv0 = (double)B.tail[TVX * B.n_rods + rod];
    const double tv1 = (double)B.tail[TVY * B.n_rods + rod];
    const double tv2 = (double)B.tail[TVZ * B.n_rods + rod];
    double qprev[9];
    for (int i = 0; i < n; ++i) {
        const int64_t s = s0 + i;
        const double v0 = S(VX, s), v1 = S(VY, s), v2 = S(VZ, s);
        Tl += 0.5 / P(P_INV_M, s) * (v0 * v0 + v1 * v1 + v2 * v2);
        double d0, d1, d2;
        if (EDGE) {
            d0 = S(RX, s); d1 = S(RY, s); d2 = S(RZ, s);
        } else {
            double rn0, rn1, rn2;
            if (i + 1 < n) { rn0 = S(RX, s + 1); rn1 = S(RY, s + 1); rn2 = S(RZ, s + 1); }
            else { rn0 = tr0; rn1 = tr1; rn2 = tr2; }
            d0 = rn0 - S(RX, s); d1 = rn1 - S(RY, s); d2 = rn2 - S(RZ, s);
        }
        const double l = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double lh = P(P_LH, s);
        const double e = l / lh;
        double q[9];
        for (int k = 0; k < 9; ++k) q[k] = S(Q00 + k, s);
        const double w0 = S(WX, s), w1 = S(WY, s), w2 = S(WZ, s);
        const double J1 = P(P_J1, s);
        Tr += 0.5 * (J1 * (w0 * w0 + w1 * w1) + 2.0 * J1 * w2 * w2) / e;
        const double sg0 = (q[0] * d0 + q[1] * d1 + q[2] * d2) / lh;
        const double sg1 = (q[3] * d0 + q[4] * d1 + q[5] * d2) / lh;
        const double sg2 = (q[6] * d0 + q[7] * d1 + q[8] * d2) / lh - 1.0;
        Us += 0.5 * (P(P_S1, s) * (sg0 * sg0 + sg1 * sg1) + P(P_S3, s) * sg2 * sg2) * lh;
        if (i > 0) {
            const int64_t sv = s - 1;   // Voronoi point i-1 lives on slot i-1
            double k0, k1, k2;
            log_relative(qprev, q, k0, k1, k2);
            const double iD = P(P_INV_DH, sv);
            k0 = k0 * iD - P(P_K0X, sv);
            k1 = k1 * iD - P(P_K0Y, sv);
            k2 = k2 * iD - P(P_K0Z, sv);
            Ub += 0.5 * (P(P_B1, sv) * (k0 * k0 + k1 * k1) + P(P_B3, sv) * k2 * k2) * P(P_DH, sv);
        }
        for (int k = 0; k < 9; ++k) qprev[k] = q[k];
        if (EDGE) { tr0 += d0; tr1 += d1; tr2 += d2; }   // anchor + edges -> node n
    }
    Tl += 0.5 / RP(R_INV_M_TAIL) * (tv0 * tv0 + tv1 * tv1 + tv2 * tv2);
    const double Wx = -(RP(R_FX) * (tr0 - RP(R_T0X)) + RP(R_FY) * (tr1 - RP(R_T0Y)) + RP(R_FZ) * (tr2 - RP(R_T0Z)));
    out[5 * rod + 0] = Tl;
    out[5 * rod + 1] = Tr;
    out[5 * rod + 2] = Us;
    out[5 * rod + 3] = Ub;
    out[5 * rod + 4] = Wx;
}

// ------------------------------------------------------------------ launchers

template <typename T, int W>
static hipError_t launch_w(const DevBatch<T> &b, int n_sub, int grid, hipStream_t s)
{
    if (grid <= 0) grid = b.n_tiles;
    hipLaunchKernelGGL((rod_step_kernel<T, W>), dim3(grid), dim3(64 * W), 0, s, b, n_sub);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_t(const DevBatch<T> &b, int waves, int n_sub, int grid, hipStream_t s)
{
    switch (waves) {
    case 1: return launch_w<T, 1>(b, n_sub, grid, s);
    case 2: return launch_w<T, 2>(b, n_sub, grid, s);
    case 4: return launch_w<T, 4>(b, n_sub, grid, s);
    case 8: return launch_w<T, 8>(b, n_sub, grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const DevBatch<double> &b, int waves, int n_sub, int grid, hipStream_t s)
{
    return launch_t<double>(b, waves, n_sub, grid, s);
}

hipError_t launch_step(const DevBatch<float> &b, int waves, int n_sub, int grid, hipStream_t s)
{
    return launch_t<float>(b, waves, n_sub, grid, s);
}

hipError_t launch_advance(int64_t *step, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step, n);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_energy_t(const DevBatch<T> &b, double *out, hipStream_t s)
{
    const int bs = 64;
    hipLaunchKernelGGL((rod_energy_kernel<T>), dim3((b.n_rods + bs - 1) / bs), dim3(bs), 0, s, b, out);
    return hipGetLastError();
}

hipError_t launch_energy(const DevBatch<double> &b, double *out, hipStream_t s)
{
    return launch_energy_t<double>(b, out, s);
}

hipError_t launch_energy(const DevBatch<float> &b, double *out, hipStream_t s)
{
    return launch_energy_t<float>(b, out, s);
}

template <typename T, int W>
static int resident_w()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rod_step_kernel<T, W>, 64 * W, 0) != hipSuccess)
        return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return per_cu * cus;
}

int step_resident_groups(int precision_f32, int waves)
{
    if (precision_f32) {
        switch (waves) {
        case 1: return resident_w<float, 1>();
        case 2: return resident_w<float, 2>();
        case 4: return resident_w<float, 4>();
        case 8: return resident_w<float, 8>();
        }
    } else {
        switch (waves) {
        case 1: return resident_w<double, 1>();
        case 2: return resident_w<double, 2>();
        case 4: return resident_w<double, 4>();
        case 8: return resident_w<double, 8>();
        }
    }
    return 0;
}

}  // namespace rodk
