// rod_kernels.hip -- gfx950 kernels of the discrete Cosserat-rod step.
//
// Mapping: one lane per element.  A workgroup of 64*W lanes owns a tile of
// whole rods laid out on consecutive lanes; lane i of a rod holds node i
// (v, and r in FP64) and element i (Q, omega, and the edge r_{i+1} - r_i in
// FP32); the rod's last lane also holds node n.  Each launch loads its
// tiles' state once, runs `n_sub` position-Verlet substeps with the state in
// registers, and stores it once.  The two-point stencils of the difference
// and averaging operators take the neighbour lane's values by DPP wave
// shifts (wave_shl:1 / wave_shr:1, full-rate VALU moves); only values that
// cross a wave boundary of a multi-wave tile go through LDS, behind one
// barrier per exchange.
//
// Model: Elastica++, Methods, "Cosserat rod dynamics", Eq. 1a (linear
// momentum) and Eq. 1b (angular momentum) on the staggered grid of nodes,
// elements and Voronoi points; time stepping per Results,
// "Performance-oriented software design" (position Verlet with the
// kinematic constraints imposed after every stage).
#include "rod.h"
#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdint>

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

// 1/sqrt(x) and 1/x from the hardware estimates (24 correct bits in both
// precisions); FP64 adds two Newton steps (24 -> 48 -> full precision).
__device__ inline double rsqrt_t(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    y = fma(0.5 * y, fma(-h, y, 1.0), y);
    h = x * y;
    return fma(0.5 * y, fma(-h, y, 1.0), y);
}
__device__ inline float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rcp_t(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ inline float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }

// DPP wave shifts: lane i reads lane i+1 (SHL) or lane i-1 (SHR) of its
// wave; the wave's edge lane reads zero.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ inline float dpp(float x)
{
    const int v = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline double dpp(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const uint32_t rlo = (uint32_t)__builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true);
    const uint32_t rhi = (uint32_t)__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)rhi << 32) | rlo);
}

// Neighbour exchange inside a tile of W waves.  `from_right` gives every
// lane the values of lane + 1, `from_left` those of lane - 1.  Called by all
// lanes (full EXEC).  For W > 1 the wave-edge values go through `lds`
// ([W][N]) behind one barrier.
template <int W, int N, typename T>
__device__ __forceinline__ void from_right(const T (&v)[N], T (&out)[N], T *lds, int wave, int wl)
{
    if constexpr (W > 1) {
        if (wl == 0) {
#pragma unroll
            for (int k = 0; k < N; ++k) lds[wave * N + k] = v[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = dpp<DPP_WAVE_SHL1>(v[k]);
    if constexpr (W > 1) {
        if (wl == 63 && wave + 1 < W) {
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = lds[(wave + 1) * N + k];
        }
    }
}

template <int W, int N, typename T>
__device__ __forceinline__ void from_left(const T (&v)[N], T (&out)[N], T *lds, int wave, int wl)
{
    if constexpr (W > 1) {
        if (wl == 63) {
#pragma unroll
            for (int k = 0; k < N; ++k) lds[wave * N + k] = v[k];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = dpp<DPP_WAVE_SHR1>(v[k]);
    if constexpr (W > 1) {
        if (wl == 0 && wave > 0) {
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = lds[(wave - 1) * N + k];
        }
    }
}

// Large-angle paths, kept out of line: they run only when a rod turns by more
// than ~0.1 rad in half a step or bends by more than ~0.06 rad between two
// elements, and inlining them would reserve their registers in the hot loop.
template <typename T>
__device__ __attribute__((noinline)) void rodrigues_coefs_general(T x, T &a, T &b)
{
    const T t = dsqrt(x);
    a = dsin(t) / t;
    b = (T(1) - dcos(t)) / x;
}

template <typename T>
__device__ __attribute__((noinline)) T log_factor_general(T s2, T c)
{
    const T s = dsqrt(s2);
    return datan2(s, c) / s;
}

// q <- exp([u]x) q for a row-major director matrix q (rows d1, d2, d3).
// exp([u]x) = I + a [u]x + b [u]x^2 with a = sin(t)/t, b = (1 - cos t)/t^2,
// t = |u|; both are even series in t^2, used for small t.  [u]x acts on the
// columns of q (the lab components of the three directors).
template <typename T>
__device__ inline void rotate_left(T q[9], T ux, T uy, T uz)
{
    const T x = ux * ux + uy * uy + uz * uz;
    // sin(t)/t = 1 - x/3! + x^2/5! - x^3/7! + x^4/9!
    T a = T(1) + x * (T(-1.0 / 6) + x * (T(1.0 / 120) + x * (T(-1.0 / 5040) + x * T(1.0 / 362880))));
    // (1-cos t)/t^2 = 1/2! - x/4! + x^2/6! - x^3/8! + x^4/10!
    T b = T(0.5) + x * (T(-1.0 / 24) + x * (T(1.0 / 720) + x * (T(-1.0 / 40320) + x * T(1.0 / 3628800))));
    if (x >= Coef<T>::rot_series_max) rodrigues_coefs_general(x, a, b);
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
// t/|w| = asin(s)/s with s = |w| when c > 0, an even series in s^2.  Lanes
// with `use` false (no Voronoi point) take the series value at s = 0, so an
// unrelated neighbour frame never sends them down the large-angle path.
template <typename T>
__device__ inline void log_relative(const T qa[9], const T qb[9], bool use, T &u0, T &u1, T &u2)
{
    auto dot = [&](int a, int b) {
        return qa[3 * a] * qb[3 * b] + qa[3 * a + 1] * qb[3 * b + 1] + qa[3 * a + 2] * qb[3 * b + 2];
    };
    const T w0 = T(0.5) * (dot(2, 1) - dot(1, 2));
    const T w1 = T(0.5) * (dot(0, 2) - dot(2, 0));
    const T w2 = T(0.5) * (dot(1, 0) - dot(0, 1));
    const T c = use ? T(0.5) * (dot(0, 0) + dot(1, 1) + dot(2, 2) - T(1)) : T(1);
    const T s2 = use ? w0 * w0 + w1 * w1 + w2 * w2 : T(0);
    // asin(s)/s = sum_k (2k)! / (4^k (k!)^2 (2k+1)) s^(2k)
    T f = T(1) + s2 * (T(1.0 / 6) + s2 * (T(3.0 / 40) + s2 * (T(5.0 / 112) + s2 * (T(35.0 / 1152)
            + s2 * (T(63.0 / 2816) + s2 * (T(231.0 / 13312) + s2 * T(143.0 / 10240)))))));
    if (!(c > T(0) && s2 < Coef<T>::log_series_max)) f = log_factor_general(s2, c);
    u0 = f * w0;
    u1 = f * w1;
    u2 = f * w2;
}

template <typename T>
__device__ inline bool finite3(T a, T b, T c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// Inclusive prefix sum of (p0, p1, p2) along each rod's lanes of a tile:
// Kogge-Stone through LDS (`sc`, 3 * 64W values), restarted where the element
// index `idx` is 0.  Its additions depend only on the element index, so every
// tile width gives the same bits.  Called by all lanes (full EXEC).
template <int W, typename T>
__device__ __forceinline__ void rod_prefix(T &p0, T &p1, T &p2, int idx, T *sc, int lane)
{
    constexpr int TL = 64 * W;
    for (int k = 1; k < TL; k <<= 1) {
        __syncthreads();
        sc[lane] = p0; sc[TL + lane] = p1; sc[2 * TL + lane] = p2;
        __syncthreads();
        if (idx >= k) {
            p0 += sc[lane - k]; p1 += sc[TL + lane - k]; p2 += sc[2 * TL + lane - k];
        }
    }
}

// Force on connected node `me` (compact index in the tile, global index g)
// from its connections: sum over them, in connection order, of
// [k (l - l0) + c dl/dt] e, e the unit vector to the partner.  `tab` holds
// rows x0 x1 x2 v0 v1 v2 of `rows` entries.  Coincident nodes exert nothing
// (the direction is undefined there).  FP64 in both precisions: the table's
// positions are FP64, and in an FP32 step the spring's small extension
// l - l0 would otherwise lose the digits of the rod-sized coordinates.
template <typename T>
__device__ inline void connection_force(const DevBatch<T> &B, const double *tab, int rows, int me, int g,
                                        double &f0, double &f1, double &f2)
{
    const int64_t E = B.conn_entries;
    const double x0 = tab[me], x1 = tab[rows + me], x2 = tab[2 * rows + me];
    const double u0 = tab[3 * rows + me], u1 = tab[4 * rows + me], u2 = tab[5 * rows + me];
    for (int e = B.conn_off[g]; e < B.conn_off[g + 1]; ++e) {
        const int p = B.conn_partner[e];
        const double dx = tab[p] - x0, dy = tab[rows + p] - x1, dz = tab[2 * rows + p] - x2;
        const double l2 = dx * dx + dy * dy + dz * dz;
        if (l2 > 0.0) {
            const double il = rsqrt_t(l2);
            const double l = l2 * il;
            const double ex = dx * il, ey = dy * il, ez = dz * il;
            const double ldot = ex * (tab[3 * rows + p] - u0) + ey * (tab[4 * rows + p] - u1) + ez * (tab[5 * rows + p] - u2);
            const double mag = B.conn_par[e] * (l - B.conn_par[2 * E + e]) + B.conn_par[E + e] * ldot;
            f0 += mag * ex; f1 += mag * ey; f2 += mag * ez;
        }
    }
}

// Contact of a node (a sphere of radius `rad` at x, velocity v) with the
// batch's planar walls: penalty normal force delta (k - c v_n) while it
// penetrates by delta = rad - (n.x - d) and that force is positive, Coulomb
// friction -mu f_n v_t / max(|v_t|, v_slip) against the tangential velocity.
// wl: the walls as (n, d) quadruples in LDS, d in the tile's frame; unrolled
// to the maximum count so that every wall's reads issue at once.
template <typename T>
__device__ inline void wall_force(const DevBatch<T> &B, const T *wl, T rad, T x0, T x1, T x2, T v0, T v1, T v2,
                                  T &f0, T &f1, T &f2)
{
#pragma unroll
    for (int w = 0; w < DEV_MAX_WALLS; ++w) {
        if (w >= B.n_walls) break;
        const T n0 = wl[4 * w], n1 = wl[4 * w + 1], n2 = wl[4 * w + 2];
        const T delta = rad - ((n0 * x0 + n1 * x1 + n2 * x2) - wl[4 * w + 3]);
        if (delta > T(0)) {
            const T vn = n0 * v0 + n1 * v1 + n2 * v2;
            const T fn = delta * (B.wall_k - B.wall_c * vn);
            if (fn > T(0)) {
                const T t0 = v0 - vn * n0, t1 = v1 - vn * n1, t2 = v2 - vn * n2;
                // 1 / max(|v_t|, v_slip) as one reciprocal square root
                const T s2 = t0 * t0 + t1 * t1 + t2 * t2, vs2 = B.wall_vslip * B.wall_vslip;
                const T g = B.wall_mu * fn * rsqrt_t(s2 > vs2 ? s2 : vs2);
                f0 += fn * n0 - g * t0;
                f1 += fn * n1 - g * t1;
                f2 += fn * n2 - g * t2;
            }
        }
    }
}

// Screen of the wall contacts of a lane: some wall within `reach` of x (the
// largest rad + reach - (n.x - d) is positive).  Branch-free over the walls,
// so that the contact forces run only in lanes near a wall.
template <typename T>
__device__ inline bool wall_reach(const DevBatch<T> &B, const T *wl, T reach, T x0, T x1, T x2)
{
    T m = T(-1);
#pragma unroll
    for (int w = 0; w < DEV_MAX_WALLS; ++w) {
        if (w < B.n_walls) {
            const T sw = reach - ((wl[4 * w] * x0 + wl[4 * w + 1] * x1 + wl[4 * w + 2] * x2) - wl[4 * w + 3]);
            m = sw > m ? sw : m;
        }
    }
    return m > T(0);
}

}  // namespace

// One launch: n_sub position-Verlet substeps for every tile (grid-stride).
//
// State per lane, in registers: the edge vector d_i = r_{i+1} - r_i, node i's
// velocity, element i's frame and angular velocity; per rod, node 0's
// position (the anchor, first lane) and node n's velocity (last lane).  The
// drift r_j += h v_j becomes d_i += h (v_{i+1} - v_i), anchor += h v_0: the
// same update in exact arithmetic, with the strains kept at the state
// precision's relative accuracy.  FP32 batches keep this form in memory too
// (absolute FP32 positions would round each drift increment against the rod's
// whole length); FP64 batches keep node positions in memory, turned into edges
// at the start of a launch and back, by a prefix sum along the rod, at its end.
//
// Voronoi point k (between elements k and k+1) belongs to lane k+1, so a
// substep needs two neighbour exchanges, each one barrier in a multi-wave
// tile: from the left, element i-1's frame, length and internal force (the
// curvature, moment and y of Voronoi point i-1, and node i's force and kick);
// from the right, Voronoi point i's moment and y and node i+1's kicked
// velocity (element i's couple and kick, and the next drift).
//
// Inside a launch the closing half drift of one step and the opening half
// drift of the next use the same velocities, so they run as one full drift
// (exp(-h/2 W) exp(-h/2 W) = exp(-h W) for one axis): a launch of S steps is
// half drift, S kicks separated by S-1 full drifts, half drift.
// Waves per SIMD: 3 (FP64, 168 VGPRs) and 5 (FP32, 96 VGPRs); FP64 tiles of 8
// waves stay at 2: their LDS admits one workgroup per CU.
#ifndef ROD_F64_WAVES_PER_SIMD
#define ROD_F64_WAVES_PER_SIMD 3
#endif
#ifndef ROD_F32_WAVES_PER_SIMD
#define ROD_F32_WAVES_PER_SIMD 5
#endif

// KIND 0: the plain step.  KIND 1: the extended step, for batches with a
// magnetic couple, gravity or muscle torques.  KIND 2: the extended step with
// rod-rod connections (connected node positions in an LDS table).  KIND 3: the
// extended step with planar walls or rod contact and connections, which needs
// every node's position in every substep (FP32: three more LDS columns).  KIND
// 4: the same without connections, their code compiled out (it held registers
// the wall and contact batches never use).
// Separate instantiations, so each kernel keeps the registers and LDS of what
// it computes.  FP32 wall and connection tiles run 3 waves per SIMD (wall
// tiles of 8 waves 2: their LDS admits one workgroup per CU); at 4 the FP32
// connection step, whose connection laws work in FP64, spilled 44 VGPRs and
// took 1.6 times as long on the 4096-bot swarm.  Each extension a batch lacks contributes an exact zero
// (zero magnetization, amplitude or gravity), so the extended kernel reproduces
// the plain one bit for bit on a plain batch.  Its multi-wave FP64 tiles and
// all its FP32 tiles run one wave per SIMD fewer than the plain step's.
template <typename T, int W, int KIND>
constexpr int step_waves_per_simd()
{
    return sizeof(T) == 8 ? ((W == 8 || (KIND > 0 && W > 1)) ? 2 : ROD_F64_WAVES_PER_SIMD)
                          : (KIND >= 3 ? (W == 8 ? 2 : ROD_F32_WAVES_PER_SIMD - 2)
                                       : KIND == 2 ? ROD_F32_WAVES_PER_SIMD - 2
                                       : KIND == 1 ? ROD_F32_WAVES_PER_SIMD - 1 : ROD_F32_WAVES_PER_SIMD);
}

template <typename T, int W, int KIND>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(step_waves_per_simd<T, W, KIND>())))
void rod_step_kernel(const DevBatch<T> B, int n_sub)
{
    constexpr bool EXT = KIND > 0;     // magnetic couple, gravity, muscle torques
    constexpr bool NODE = KIND >= 2;   // and node interactions (connections, walls)
    constexpr bool WALL = KIND >= 3;   // planar walls or rod contact: every node's position
    constexpr bool CONN = KIND == 2 || KIND == 3;   // connections (compiled out of KIND 4)
    constexpr bool POS = sizeof(T) == 8;   // node positions in memory
    constexpr int TL = 64 * W;
    constexpr int NA = 13;     // from the left: frame (9), length, internal force (3)
    constexpr int NB = 9;      // from the right: Voronoi moment (3), y (3), node velocity (3)
    constexpr int NL = W > 1 ? W : 1;
    // lane-private constants (each lane reads back only its own column, so no
    // barrier is needed): a register extension for values used once a substep.
    // The Voronoi quantities of a lane are those of the point on its left.
    enum { C_J1, C_INV_J1, C_DH, C_INV_DH, C_B1, C_B3, C_K0X, C_K0Y, C_K0Z, C_GAMMA,
           C_INV_MT, C_FX, C_FY, C_FZ, C_CX, C_CY, C_CZ, C_INV_M, C_LH, C_INV_LH, C_S1, C_S3,
           C_MX, C_MY, C_MZ,     // magnetization times rest length (EXT only)
           C_AX, C_AY, C_AZ,     // muscle amplitude times axis (EXT only)
           C_RAD,                // rod radius (KIND 3, 4)
           C_PX, C_PY, C_PZ };   // node i's position (KIND 3, 4, FP32; FP64 has it in registers)
    constexpr int N_C = WALL ? (POS ? C_RAD + 1 : C_PZ + 1) : (EXT ? C_AZ + 1 : C_MX);
    // One LDS block in a fixed order: the small wave-edge exchange buffers first,
    // so their addresses fit the 8-bit offsets of ds_write2/ds_read2 and need no
    // per-access address arithmetic, then the constant columns.
    struct Shared {
        T lxa[NL * NA];            // wave-edge values of the two exchanges
        T lxb[NL * NB];
        double phs[2 * TL];        // couple phase increment: sin, cos
        double mph[EXT ? 2 * TL : 1];   // muscle phase increment: sin, cos (EXT only)
        T wls[WALL ? 4 * DEV_MAX_WALLS : 1];   // walls (n, d), d in the tile's frame (KIND 3, 4)
        T cst[N_C * TL];
    };
    __shared__ Shared sh;
    // connections: rows x0 x1 x2 v0 v1 v2 (FP64) of the tile's connected
    // nodes; for FP32, also the scratch of the prefix sum of node positions at
    // the tile's start (FP64 with connections, else FP32); sized at launch
    extern __shared__ __align__(16) unsigned char conn_lds[];
    double *const tab = reinterpret_cast<double *>(conn_lds);
    T *const lxa = sh.lxa, *const lxb = sh.lxb;
    T *const cst = sh.cst;
    double *const phs = sh.phs;

    const int lane = threadIdx.x;
    const int wave = lane >> 6, wl = lane & 63;
    const int64_t NS = B.n_slots;
    const int64_t step0 = *B.step;
    const T h = T(B.dt);
    const T hh = T(0.5 * B.dt);

    const int n_work = B.tile_list ? B.n_list : B.n_tiles;
    for (int it = blockIdx.x; it < n_work; it += gridDim.x) {
        const int tile = B.tile_list ? B.tile_list[it] : it;
        const int64_t s = (int64_t)tile * TL + lane;
        const int rod = B.slot_rod[s];
        const bool valid = rod >= 0;
        const int rr = valid ? rod : 0;
        const int i = B.slot_idx[s];
        const int n = valid ? B.rod_n[rr] : 1;
        const int flags = valid ? B.rod_flags[rr] : 0;
        const bool last = valid && (i == n - 1);
        const bool first = i == 0;
        const bool hasl = valid && i > 0;    // Voronoi point i-1 exists
        const bool fix0 = first && (flags & FLAG_CLAMP0);
        const bool fix1 = last && (flags & FLAG_CLAMP1);
        // rods switched off by the caller keep their state; a tile with none
        // active is skipped (uniform across the workgroup)
        const bool act = valid && (!B.active || B.active[rr]);
        if (!__syncthreads_or(act)) continue;
        // kinematic constraints as kick factors: a clamped node or element
        // starts at rest and never receives an increment
        const T hv = fix0 ? T(0) : h;
        const T hw = (fix0 || fix1) ? T(0) : h;
        const T hu = fix1 ? T(0) : h;

        // ---- constants: all in this lane's LDS column (registers hold the state
        // and the substep's temporaries); set up before the state is loaded, so
        // the phase computations have the registers to themselves
        const T *pp = B.param + s;
        double ps = 0.0, pc = 1.0;
        {
            T *cw = cst + lane;
            const T lh = pp[P_LH * NS];
            cw[C_INV_M * TL] = pp[P_INV_M * NS];
            cw[C_LH * TL] = lh;
            cw[C_INV_LH * TL] = pp[P_INV_LH * NS];
            cw[C_S1 * TL] = pp[P_S1 * NS];
            cw[C_S3 * TL] = pp[P_S3 * NS];
            const T J1 = pp[P_J1 * NS];
            cw[C_J1 * TL] = J1;
            cw[C_INV_J1 * TL] = T(1) / J1;
            cw[C_DH * TL] = pp[P_DH * NS];
            cw[C_INV_DH * TL] = pp[P_INV_DH * NS];
            // no Voronoi point left of a rod's first element: zero stiffness there
            cw[C_B1 * TL] = hasl ? pp[P_B1 * NS] : T(0);
            cw[C_B3 * TL] = hasl ? pp[P_B3 * NS] : T(0);
            cw[C_K0X * TL] = pp[P_K0X * NS];
            cw[C_K0Y * TL] = pp[P_K0Y * NS];
            cw[C_K0Z * TL] = pp[P_K0Z * NS];
            cw[C_GAMMA * TL] = B.rodp[R_GAMMA * B.n_rods + rr];
            cw[C_INV_MT * TL] = last ? B.rodp[R_INV_M_TAIL * B.n_rods + rr] : T(0);
            cw[C_FX * TL] = last ? B.rodp[R_FX * B.n_rods + rr] : T(0);
            cw[C_FY * TL] = last ? B.rodp[R_FY * B.n_rods + rr] : T(0);
            cw[C_FZ * TL] = last ? B.rodp[R_FZ * B.n_rods + rr] : T(0);
            // distributed couple amplitude times rest length; its time factor
            // sin(2 pi f t + phi) at the substep midpoints by rotation recurrence
            T c0 = 0, c1 = 0, c2 = 0;
            double ds = 0.0, dc = 1.0;
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
            cw[C_CX * TL] = c0;
            cw[C_CY * TL] = c1;
            cw[C_CZ * TL] = c2;
            phs[lane] = ds;
            phs[TL + lane] = dc;
        }
        // extended step: magnetization and muscle amplitude columns; the
        // field's phase 2 pi f t (the same for every lane) and the muscle
        // wave's phase 2 pi f_r t - q_r s_k + phi_r at the substep midpoints,
        // both advanced by rotation recurrences
        double fs = 0.0, fc = 1.0, ms = 0.0, mc = 1.0;
        if constexpr (EXT) {
            T *cw = cst + lane;
            const bool hm = B.mag != nullptr, ha = B.mus != nullptr && valid;
            cw[C_MX * TL] = hm ? B.mag[s] : T(0);
            cw[C_MY * TL] = hm ? B.mag[NS + s] : T(0);
            cw[C_MZ * TL] = hm ? B.mag[2 * NS + s] : T(0);
            cw[C_AX * TL] = ha ? B.mus[s] : T(0);
            cw[C_AY * TL] = ha ? B.mus[NS + s] : T(0);
            cw[C_AZ * TL] = ha ? B.mus[2 * NS + s] : T(0);
            const double tm = B.t0 + ((double)step0 + 0.5) * B.dt;
            if (hm) {
                const double ph = 2.0 * M_PI * B.field_freq * tm;
                fs = sin(ph);
                fc = cos(ph);
            }
            double mds = 0.0, mdc = 1.0;
            if (ha) {
                const double fr = B.mus_freq[rr];
                const double ph = 2.0 * M_PI * fr * tm + B.mus_ofs[s];
                ms = sin(ph);
                mc = cos(ph);
                const double dp = 2.0 * M_PI * fr * B.dt;
                mds = sin(dp);
                mdc = cos(dp);
            }
            sh.mph[lane] = mds;
            sh.mph[TL + lane] = mdc;
        }

        // ---- state: d = edge i (FP64: node i's position until the first
        // exchange), v = node i, t = anchor (first lane; FP64: node n's position
        // on the last lane until the first exchange), u = node n (last lane)
        const T *st = B.state + s;
        T d0 = st[RX * NS], d1 = st[RY * NS], d2 = st[RZ * NS];
        T v0 = st[VX * NS], v1 = st[VY * NS], v2 = st[VZ * NS];
        T q[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) q[k] = st[(Q00 + k) * NS];
        T w0 = st[WX * NS], w1 = st[WY * NS], w2 = st[WZ * NS];
        T t0 = 0, t1 = 0, t2 = 0, u0 = 0, u1 = 0, u2 = 0;
        if (POS ? last : (valid && first)) {
            t0 = B.tail[TRX * B.n_rods + rr]; t1 = B.tail[TRY * B.n_rods + rr]; t2 = B.tail[TRZ * B.n_rods + rr];
        }
        if (last) {
            u0 = B.tail[TVX * B.n_rods + rr]; u1 = B.tail[TVY * B.n_rods + rr]; u2 = B.tail[TVZ * B.n_rods + rr];
        }
        // velocity of node i+1 (refreshed by every kick's exchange)
        T vn0, vn1, vn2;
        if constexpr (POS) {
            // and node i+1's position: edge i, with node i's position as the anchor
            const T a0[6] = {v0, v1, v2, d0, d1, d2};
            T b0[6];
            from_right<W>(a0, b0, lxb, wave, wl);
            vn0 = last ? u0 : b0[0]; vn1 = last ? u1 : b0[1]; vn2 = last ? u2 : b0[2];
            const T rn0 = last ? t0 : b0[3], rn1 = last ? t1 : b0[4], rn2 = last ? t2 : b0[5];
            t0 = d0; t1 = d1; t2 = d2;
            d0 = rn0 - t0; d1 = rn1 - t1; d2 = rn2 - t2;
        } else {
            const T a0[3] = {v0, v1, v2};
            T b0[3];
            from_right<W>(a0, b0, lxb, wave, wl);
            vn0 = last ? u0 : b0[0]; vn1 = last ? u1 : b0[1]; vn2 = last ? u2 : b0[2];
        }

        // node interactions: node positions (in the frame of the tile's first
        // rod) into this lane's LDS columns, and the connected nodes' into the
        // connection table
        int ci = -1, cn = -1, cbase = 0;
        if constexpr (NODE) {
            T x0, x1, x2;
            double X0, X1, X2;   // the same in FP64, for the connection table
            if constexpr (POS) {
                x0 = t0; x1 = t1; x2 = t2;   // node i's position
                X0 = x0; X1 = x1; X2 = x2;
            } else {
                // rod origin + anchor + the edges before node i (a prefix sum
                // along the rod; in FP64 when the tile has connections)
                const T e3[3] = {d0, d1, d2};
                T lf[3];
                from_left<W>(e3, lf, lxa, wave, wl);
                if (CONN && B.conn_idx) {
                    X0 = first ? B.rod_org[rr] + (double)t0 : (double)lf[0];
                    X1 = first ? B.rod_org[B.n_rods + rr] + (double)t1 : (double)lf[1];
                    X2 = first ? B.rod_org[2 * B.n_rods + rr] + (double)t2 : (double)lf[2];
                    rod_prefix<W>(X0, X1, X2, i, tab, lane);
                    x0 = T(X0); x1 = T(X1); x2 = T(X2);
                } else {
                    x0 = first ? T(B.rod_org[rr]) + t0 : lf[0];
                    x1 = first ? T(B.rod_org[B.n_rods + rr]) + t1 : lf[1];
                    x2 = first ? T(B.rod_org[2 * B.n_rods + rr]) + t2 : lf[2];
                    rod_prefix<W>(x0, x1, x2, i, reinterpret_cast<T *>(conn_lds), lane);
                    X0 = x0; X1 = x1; X2 = x2;
                }
                __syncthreads();
            }
            // positions after the opening half drift
            if constexpr (WALL) {
                if (lane < 4 * B.n_walls) {
                    const int w = lane >> 2, a = lane & 3;
                    sh.wls[lane] = a < 3 ? B.wall[w][a] : B.wall_off[8 * (int64_t)tile + w];
                }
                // every wave reads all walls (the previous tile's last reads
                // are behind the barrier of its last exchange B)
                __syncthreads();
                T *cw = cst + lane;
                cw[C_RAD * TL] = valid ? T(B.rod_rad[rr]) : T(0);
                if constexpr (!POS) {
                    cw[C_PX * TL] = x0 + hh * v0; cw[C_PY * TL] = x1 + hh * v1; cw[C_PZ * TL] = x2 + hh * v2;
                }
            }
            if (CONN && B.conn_idx) {
                const int rows = B.conn_nodes;
                ci = B.conn_idx[s];
                cn = last ? B.conn_idx[NS + s] : -1;
                cbase = B.conn_tbase[tile];
                const double H = hh;
                if (ci >= 0) { tab[ci] = X0 + H * v0; tab[rows + ci] = X1 + H * v1; tab[2 * rows + ci] = X2 + H * v2; }
                if (cn >= 0) {
                    tab[cn] = X0 + d0 + H * u0; tab[rows + cn] = X1 + d1 + H * u1; tab[2 * rows + cn] = X2 + d2 + H * u2;
                }
            }
        }

        // ---- opening half drift (constraints hold: clamped v, omega are zero)
        d0 += hh * (vn0 - v0); d1 += hh * (vn1 - v1); d2 += hh * (vn2 - v2);
        t0 += hh * v0; t1 += hh * v1; t2 += hh * v2;
        rotate_left(q, -hh * w0, -hh * w1, -hh * w2);

        for (int sub = 0; sub < n_sub; ++sub) {
            // the lane-private constants are re-read every substep: an opaque
            // address keeps the compiler from hoisting them into registers
            int cofs = lane;
            asm volatile("" : "+v"(cofs));
            const T *cl = cst + cofs;
            const double *phl = phs + cofs;

            // ---- kinematics, shear/stretch strain and internal force of element i
            const T lh = cl[C_LH * TL], inv_lh = cl[C_INV_LH * TL];
            const T S1 = cl[C_S1 * TL], S3 = cl[C_S3 * TL];
            const T l2 = d0 * d0 + d1 * d1 + d2 * d2;
            const T inv_l = rsqrt_t(l2);
            const T l = l2 * inv_l;
            const T e = l * inv_lh;
            const T inv_e = lh * inv_l;
            const T edot = ((d0 * (vn0 - v0) + d1 * (vn1 - v1) + d2 * (vn2 - v2)) * inv_l) * inv_lh;
            // sigma = Q d / lh - e3
            const T sg0 = (q[0] * d0 + q[1] * d1 + q[2] * d2) * inv_lh;
            const T sg1 = (q[3] * d0 + q[4] * d1 + q[5] * d2) * inv_lh;
            const T sg2 = (q[6] * d0 + q[7] * d1 + q[8] * d2) * inv_lh - T(1);
            const T ss0 = S1 * sg0, ss1 = S1 * sg1, ss2 = S3 * sg2;
            // internal force n = Q^T S sigma / e (lab)
            const T nf0 = (q[0] * ss0 + q[3] * ss1 + q[6] * ss2) * inv_e;
            const T nf1 = (q[1] * ss0 + q[4] * ss1 + q[7] * ss2) * inv_e;
            const T nf2 = (q[2] * ss0 + q[5] * ss1 + q[8] * ss2) * inv_e;

            // ---- exchange A: element i-1's frame, length and internal force.
            // A rod's first lane sits next to the previous rod's last lane or
            // at the tile edge (zeros): its Voronoi stiffness is zero and its
            // left force is masked.
            T M0, M1, M2, y0, y1, y2, np0, np1, np2;
            {
                const T aa[NA] = {q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], l, nf0, nf1, nf2};
                T ba[NA];
                from_left<W>(aa, ba, lxa, wave, wl);
                // curvature of Voronoi point i-1: log(Q_{i-1} Q_i^T) / Dh
                T k0, k1, k2;
                log_relative(ba, q, hasl, k0, k1, k2);
                const T inv_Dh = cl[C_INV_DH * TL], Dh = cl[C_DH * TL];
                k0 *= inv_Dh; k1 *= inv_Dh; k2 *= inv_Dh;
                const T eps = (ba[9] + l) * (T(0.5) * inv_Dh);
                const T ie3 = rcp_t(eps * eps * eps);
                M0 = cl[C_B1 * TL] * (k0 - cl[C_K0X * TL]) * ie3;
                M1 = cl[C_B1 * TL] * (k1 - cl[C_K0Y * TL]) * ie3;
                M2 = cl[C_B3 * TL] * (k2 - cl[C_K0Z * TL]) * ie3;
                if constexpr (EXT) {
                    // active muscle moment, part of the internal moment
                    const T sa = T(ms);
                    M0 += cl[C_AX * TL] * sa;
                    M1 += cl[C_AY * TL] * sa;
                    M2 += cl[C_AZ * TL] * sa;
                }
                y0 = (k1 * M2 - k2 * M1) * Dh;
                y1 = (k2 * M0 - k0 * M2) * Dh;
                y2 = (k0 * M1 - k1 * M0) * Dh;
                np0 = first ? T(0) : ba[10];
                np1 = first ? T(0) : ba[11];
                np2 = first ? T(0) : ba[12];
            }

            // ---- connection forces on node i and node n (pre-kick velocities)
            T fc0 = 0, fc1 = 0, fc2 = 0, gc0 = 0, gc1 = 0, gc2 = 0;
            if constexpr (NODE) {
                if (CONN && B.conn_idx) {
                    const int rows = B.conn_nodes;
                    if (ci >= 0) { tab[3 * rows + ci] = v0; tab[4 * rows + ci] = v1; tab[5 * rows + ci] = v2; }
                    if (cn >= 0) { tab[3 * rows + cn] = u0; tab[4 * rows + cn] = u1; tab[5 * rows + cn] = u2; }
                    __syncthreads();
                    double f0 = 0, f1 = 0, f2 = 0, g0 = 0, g1 = 0, g2 = 0;
                    if (ci >= 0) connection_force(B, tab, rows, ci, cbase + ci, f0, f1, f2);
                    if (cn >= 0) connection_force(B, tab, rows, cn, cbase + cn, g0, g1, g2);
                    fc0 = T(f0); fc1 = T(f1); fc2 = T(f2);
                    gc0 = T(g0); gc1 = T(g1); gc2 = T(g2);
                }
                if constexpr (WALL) {
                    // node i at x, node n (last lane) at x + the edge
                    const T rad = cl[C_RAD * TL];
                    T x0, x1, x2;
                    if constexpr (POS) {
                        x0 = t0; x1 = t1; x2 = t2;
                    } else {
                        x0 = cl[C_PX * TL]; x1 = cl[C_PY * TL]; x2 = cl[C_PZ * TL];
                    }
                    // node n lies within |d| = l of node i: on a rod's last
                    // lane one screen covers both (up to the rounding of the
                    // positions)
                    if (wall_reach(B, sh.wls, last ? rad + l : rad, x0, x1, x2)) {
                        wall_force(B, sh.wls, rad, x0, x1, x2, v0, v1, v2, fc0, fc1, fc2);
                        if (last) wall_force(B, sh.wls, rad, x0 + d0, x1 + d1, x2 + d2, u0, u1, u2, gc0, gc1, gc2);
                    }
                    // rod-rod contact, from the contact pass before this
                    // launch (one step per launch)
                    if (B.cforce) {
                        const int64_t NN = B.n_slots + B.n_rods;
                        const int64_t sl = (int64_t)tile * TL + lane;
                        fc0 += T(B.cforce[sl]); fc1 += T(B.cforce[NN + sl]); fc2 += T(B.cforce[2 * NN + sl]);
                        if (last) {
                            const int64_t id = B.n_slots + B.slot_rod[sl];
                            gc0 += T(B.cforce[id]); gc1 += T(B.cforce[NN + id]); gc2 += T(B.cforce[2 * NN + id]);
                        }
                    }
                }
            }

            // ---- Eq. 1a at node i (and node n on the last lane); kick
            const T gamma = cl[C_GAMMA * TL];
            {
                const T inv_m = cl[C_INV_M * TL];
                T a0 = (nf0 - np0) * inv_m - gamma * v0;
                T a1 = (nf1 - np1) * inv_m - gamma * v1;
                T a2 = (nf2 - np2) * inv_m - gamma * v2;
                const T inv_mt = cl[C_INV_MT * TL];
                T b0 = (cl[C_FX * TL] - nf0) * inv_mt - gamma * u0;
                T b1 = (cl[C_FY * TL] - nf1) * inv_mt - gamma * u1;
                T b2 = (cl[C_FZ * TL] - nf2) * inv_mt - gamma * u2;
                if constexpr (EXT) {
                    a0 += B.grav[0] + fc0 * inv_m; a1 += B.grav[1] + fc1 * inv_m; a2 += B.grav[2] + fc2 * inv_m;
                    b0 += B.grav[0] + gc0 * inv_mt; b1 += B.grav[1] + gc1 * inv_mt; b2 += B.grav[2] + gc2 * inv_mt;
                }
                v0 += hv * a0; v1 += hv * a1; v2 += hv * a2;
                u0 += hu * b0; u1 += hu * b1; u2 += hu * b2;
            }

            // ---- exchange B: Voronoi point i's moment and y, node i+1's kicked velocity
            T mr0, mr1, mr2, yr0, yr1, yr2;
            {
                const T ab[NB] = {M0, M1, M2, y0, y1, y2, v0, v1, v2};
                T bb[NB];
                from_right<W>(ab, bb, lxb, wave, wl);
                mr0 = bb[0]; mr1 = bb[1]; mr2 = bb[2];
                yr0 = bb[3]; yr1 = bb[4]; yr2 = bb[5];
                vn0 = last ? u0 : bb[6]; vn1 = last ? u1 : bb[7]; vn2 = last ? u2 : bb[8];
            }

            // ---- Eq. 1b at element i (pre-kick omega, e and edot)
            // Q t = (sigma + e3) / e
            const T qt0 = sg0 * inv_e, qt1 = sg1 * inv_e, qt2 = (sg2 + T(1)) * inv_e;
            const T J1 = cl[C_J1 * TL];
            const T jw0 = J1 * w0 * inv_e, jw1 = J1 * w1 * inv_e, jw2 = T(2) * J1 * w2 * inv_e;
            const T ede = edot * inv_e;
            const T cs = T(ps);
            const T tq0 = (mr0 - M0) + T(0.5) * (y0 + yr0) + (qt1 * ss2 - qt2 * ss1) * lh
                        + (jw1 * w2 - jw2 * w1) + jw0 * ede + cl[C_CX * TL] * cs;
            const T tq1 = (mr1 - M1) + T(0.5) * (y1 + yr1) + (qt2 * ss0 - qt0 * ss2) * lh
                        + (jw2 * w0 - jw0 * w2) + jw1 * ede + cl[C_CY * TL] * cs;
            const T tq2 = (mr2 - M2) + T(0.5) * (y2 + yr2) + (qt0 * ss1 - qt1 * ss0) * lh
                        + (jw0 * w1 - jw1 * w0) + jw2 * ede + cl[C_CZ * TL] * cs;
            T mc0 = 0, mc1 = 0, mc2 = 0;
            if constexpr (EXT) {
                // magnetic couple (m lh) x (Q b(t)), material frame
                const T cb = T(fc), sb = T(fs);
                const T b0 = B.field[0] + B.field[3] * cb + B.field[6] * sb;
                const T b1 = B.field[1] + B.field[4] * cb + B.field[7] * sb;
                const T b2 = B.field[2] + B.field[5] * cb + B.field[8] * sb;
                const T qb0 = q[0] * b0 + q[1] * b1 + q[2] * b2;
                const T qb1 = q[3] * b0 + q[4] * b1 + q[5] * b2;
                const T qb2 = q[6] * b0 + q[7] * b1 + q[8] * b2;
                const T m0 = cl[C_MX * TL], m1 = cl[C_MY * TL], m2 = cl[C_MZ * TL];
                mc0 = m1 * qb2 - m2 * qb1;
                mc1 = m2 * qb0 - m0 * qb2;
                mc2 = m0 * qb1 - m1 * qb0;
            }
            const T eJ = e * cl[C_INV_J1 * TL];
            const T al0 = eJ * (tq0 + mc0) - gamma * w0;
            const T al1 = eJ * (tq1 + mc1) - gamma * w1;
            const T al2 = T(0.5) * eJ * (tq2 + mc2) - gamma * w2;
            w0 += hw * al0; w1 += hw * al1; w2 += hw * al2;

            // ---- drift: full between two kicks of this launch, half after the last
            const T dd = sub + 1 < n_sub ? h : hh;
            d0 += dd * (vn0 - v0); d1 += dd * (vn1 - v1); d2 += dd * (vn2 - v2);
            t0 += dd * v0; t1 += dd * v1; t2 += dd * v2;
            if constexpr (NODE) {
                if constexpr (WALL && !POS) {
                    T *cw = cst + cofs;
                    cw[C_PX * TL] += dd * v0; cw[C_PY * TL] += dd * v1; cw[C_PZ * TL] += dd * v2;
                }
                if (CONN && B.conn_idx) {
                    const int rows = B.conn_nodes;
                    const double D = dd;
                    if (ci >= 0) { tab[ci] += D * v0; tab[rows + ci] += D * v1; tab[2 * rows + ci] += D * v2; }
                    if (cn >= 0) { tab[cn] += D * u0; tab[rows + cn] += D * u1; tab[2 * rows + cn] += D * u2; }
                }
            }
            rotate_left(q, -dd * w0, -dd * w1, -dd * w2);

            // advance the couple's phase by one step
            {
                const double ds = phl[0], dc = phl[TL];
                const double nps = ps * dc + pc * ds;
                pc = pc * dc - ps * ds;
                ps = nps;
            }
            if constexpr (EXT) {
                const double nfs = fs * B.field_dc + fc * B.field_ds;
                fc = fc * B.field_dc - fs * B.field_ds;
                fs = nfs;
                const double mds = sh.mph[cofs], mdc = sh.mph[TL + cofs];
                const double nms = ms * mdc + mc * mds;
                mc = mc * mdc - ms * mds;
                ms = nms;
            }
        }

        // per-slot facts re-read through an opaque slot index instead of being
        // kept (and spilled) across the substep loop
        int64_t s_out = s;
        asm volatile("" : "+v"(s_out));
        const int rod_o = B.slot_rod[s_out];
        const bool valid_o = rod_o >= 0;
        const int rr_o = valid_o ? rod_o : 0;
        const int i_o = B.slot_idx[s_out];
        const bool first_o = i_o == 0;
        const bool last_o = valid_o && i_o == B.rod_n[rr_o] - 1;
        const bool act_o = valid_o && (!B.active || B.active[rr_o]);
        if constexpr (POS) {
            // node positions from the edges, r_i = anchor + d_0 + ... + d_{i-1}:
            // a prefix sum along the rod (Kogge-Stone over the tile's lanes in
            // LDS, restarted at each rod's first lane; its additions depend only
            // on the element index, so every tile width gives the same bits).
            // Afterwards d holds node i's position and t node n's (last lane).
            // Launches of a few substeps (contact batches take one) skip the sum:
            // t, node i's position drifted with v_i, differs from the edges' sum
            // by a few roundings only, and the sum's barriers cost about as much
            // as the substep itself.  (n_sub is the same for the whole grid.)
            if (n_sub <= 4) {
                const T n0 = t0 + d0, n1 = t1 + d1, n2 = t2 + d2;
                d0 = t0; d1 = t1; d2 = t2;
                t0 = n0; t1 = n1; t2 = n2;
            } else {
                const T e3[3] = {d0, d1, d2};
                T lf[3];
                from_left<W>(e3, lf, lxa, wave, wl);
                T p0 = first_o ? t0 : lf[0], p1 = first_o ? t1 : lf[1], p2 = first_o ? t2 : lf[2];
                T *const sc = cst;   // the constant columns are not read any more
                for (int k = 1; k < TL; k <<= 1) {
                    __syncthreads();
                    sc[lane] = p0; sc[TL + lane] = p1; sc[2 * TL + lane] = p2;
                    __syncthreads();
                    if (i_o >= k) {
                        p0 += sc[lane - k]; p1 += sc[TL + lane - k]; p2 += sc[2 * TL + lane - k];
                    }
                }
                t0 = p0 + d0; t1 = p1 + d1; t2 = p2 + d2;
                d0 = p0; d1 = p1; d2 = p2;
            }
        }

        if (act_o) {
            T *so = B.state + s_out;
            so[RX * NS] = d0; so[RY * NS] = d1; so[RZ * NS] = d2;
            so[VX * NS] = v0; so[VY * NS] = v1; so[VZ * NS] = v2;
#pragma unroll
            for (int k = 0; k < 9; ++k) so[(Q00 + k) * NS] = q[k];
            so[WX * NS] = w0; so[WY * NS] = w1; so[WZ * NS] = w2;
            bool ok = finite3(d0, d1, d2) && finite3(v0, v1, v2) && finite3(w0, w1, w2)
                    && finite3(q[0], q[1], q[2]) && finite3(q[3], q[4], q[5]) && finite3(q[6], q[7], q[8]);
            if (POS ? last_o : first_o) {
                B.tail[TRX * B.n_rods + rr_o] = t0; B.tail[TRY * B.n_rods + rr_o] = t1; B.tail[TRZ * B.n_rods + rr_o] = t2;
                ok = ok && finite3(t0, t1, t2);
            }
            if (last_o) {
                B.tail[TVX * B.n_rods + rr_o] = u0; B.tail[TVY * B.n_rods + rr_o] = u1; B.tail[TVZ * B.n_rods + rr_o] = u2;
                ok = ok && finite3(u0, u1, u2);
            }
            if (!ok) atomicOr(&B.nonfinite[rr_o], ROD_FLAG_NONFINITE);   // keeps the other flag bits
        }
        if constexpr (W > 1) __syncthreads();   // LDS reuse by the next tile
    }
}

__global__ void advance_kernel(int64_t *step, int64_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += n;
}

__global__ void set_step_kernel(int64_t *step, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step = v;
}

// Position of a connected node in the frame of its tile's first rod (FP64:
// the stored positions; FP32: rod origin + anchor + the edges before it, in
// FP64).  col 0: the slot's node i; col 1: node n of the rod ending there.
template <typename T>
__device__ void conn_node_position(const DevBatch<T> &B, int64_t slot, int col, double x[3])
{
    constexpr bool EDGE = sizeof(T) == 4;
    const int64_t NS = B.n_slots;
    const int rod = B.slot_rod[slot];
    if (!EDGE) {
        for (int a = 0; a < 3; ++a)
            x[a] = col == 0 ? (double)B.state[(RX + a) * NS + slot] : (double)B.tail[(TRX + a) * B.n_rods + rod];
        return;
    }
    const int j = B.slot_idx[slot] + col;
    const int64_t s0 = B.rod_slot[rod];
    for (int a = 0; a < 3; ++a) {
        double v = (double)B.rod_org[a * B.n_rods + rod] + (double)B.tail[(TRX + a) * B.n_rods + rod];
        for (int k = 0; k < j; ++k) v += (double)B.state[(RX + a) * NS + s0 + k];
        x[a] = v;
    }
}

// Per-rod energies, one thread per rod walking its slots (off the step path).
// FP32 batches hold edge vectors: node n = anchor + sum of edges (in FP64).
template <typename T>
__global__ void rod_energy_kernel(const DevBatch<T> B, double *out, const int32_t *map, int n_map)
{
    constexpr bool EDGE = sizeof(T) == 4;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;   // output row: rod `row`, or rod map[row]
    if (row >= (map ? n_map : B.n_rods)) return;
    const int rod = map ? map[row] : row;
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
    const double g0 = (double)B.grav[0], g1 = (double)B.grav[1], g2 = (double)B.grav[2];
    const bool grav = B.ext && B.grav_r0;
    const int64_t NT = NS + B.n_rods;
    double Wg = 0;   // g . sum_j m_j (r_j - r_j(0))
    for (int i = 0; i < n; ++i) {
        const int64_t s = s0 + i;
        const double v0 = S(VX, s), v1 = S(VY, s), v2 = S(VZ, s);
        Tl += 0.5 / P(P_INV_M, s) * (v0 * v0 + v1 * v1 + v2 * v2);
        if (grav) {
            const double x0 = (EDGE ? tr0 : S(RX, s)) - B.grav_r0[s];
            const double x1 = (EDGE ? tr1 : S(RY, s)) - B.grav_r0[NT + s];
            const double x2 = (EDGE ? tr2 : S(RZ, s)) - B.grav_r0[2 * NT + s];
            Wg += (g0 * x0 + g1 * x1 + g2 * x2) / P(P_INV_M, s);
        }
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
            const int64_t sv = s;       // Voronoi point i-1 lives on slot i
            double k0, k1, k2;
            log_relative(qprev, q, true, k0, k1, k2);
            const double iD = P(P_INV_DH, sv);
            k0 = k0 * iD - P(P_K0X, sv);
            k1 = k1 * iD - P(P_K0Y, sv);
            k2 = k2 * iD - P(P_K0Z, sv);
            Ub += 0.5 * (P(P_B1, sv) * (k0 * k0 + k1 * k1) + P(P_B3, sv) * k2 * k2) * P(P_DH, sv);
        }
        for (int k = 0; k < 9; ++k) qprev[k] = q[k];
        if (EDGE) { tr0 += d0; tr1 += d1; tr2 += d2; }   // anchor + edges -> node i+1
    }
    Tl += 0.5 / RP(R_INV_M_TAIL) * (tv0 * tv0 + tv1 * tv1 + tv2 * tv2);
    double Wx = -(RP(R_FX) * (tr0 - RP(R_T0X)) + RP(R_FY) * (tr1 - RP(R_T0Y)) + RP(R_FZ) * (tr2 - RP(R_T0Z)));
    if (grav) {
        const int64_t c = NS + rod;
        Wg += (g0 * (tr0 - B.grav_r0[c]) + g1 * (tr1 - B.grav_r0[NT + c]) + g2 * (tr2 - B.grav_r0[2 * NT + c]))
            / RP(R_INV_M_TAIL);
        Wx -= Wg;
    }
    if (B.ext && B.n_walls) {
        // penalty potential 1/2 k delta^2 of every node in contact with a wall
        const double rad = (double)B.rod_rad[rod];
        const T *woff = B.wall_off + 8 * (s0 / (NS / B.n_tiles));
        for (int j = 0; j <= n; ++j) {
            double x[3];
            const int64_t slot = s0 + (j < n ? j : n - 1);
            conn_node_position(B, slot, j < n ? 0 : 1, x);
            for (int w = 0; w < B.n_walls; ++w) {
                const double delta = rad - ((double)B.wall[w][0] * x[0] + (double)B.wall[w][1] * x[1]
                                            + (double)B.wall[w][2] * x[2] - (double)woff[w]);
                if (delta > 0) Wx += 0.5 * (double)B.wall_k * delta * delta;
            }
        }
    }
    if (B.ext && B.conn_idx) {
        // half of the potential 1/2 k (l - l0)^2 of every connection at this rod's nodes
        const int64_t TLn = NS / B.n_tiles;
        const int64_t E = B.conn_entries;
        for (int j = 0; j <= n; ++j) {
            const int col = j < n ? 0 : 1;
            const int64_t slot = s0 + (j < n ? j : n - 1);
            const int me = B.conn_idx[col * NS + slot];
            if (me < 0) continue;
            const int tb = B.conn_tbase[slot / TLn];
            double x[3];
            conn_node_position(B, slot, col, x);
            for (int e = B.conn_off[tb + me]; e < B.conn_off[tb + me + 1]; ++e) {
                const int key = B.conn_key[tb + B.conn_partner[e]];
                double xp[3];
                conn_node_position(B, key / 2, key % 2, xp);
                const double l = sqrt((xp[0] - x[0]) * (xp[0] - x[0]) + (xp[1] - x[1]) * (xp[1] - x[1])
                                      + (xp[2] - x[2]) * (xp[2] - x[2]));
                const double ext = l - (double)B.conn_par[2 * E + e];
                Wx += 0.25 * (double)B.conn_par[e] * ext * ext;
            }
        }
    }
    out[5 * row + 0] = Tl;
    out[5 * row + 1] = Tr;
    out[5 * row + 2] = Us;
    out[5 * row + 3] = Ub;
    if (B.cpot) {
        // rod-rod contact: the nodes' shares of the pairs' potentials
        for (int i = 0; i < n; ++i) Wx += B.cpot[s0 + i];
        Wx += B.cpot[NS + rod];
    }
    out[5 * row + 4] = Wx;
}

// ------------------------------------------------------------------ launchers

// Dynamic LDS of the node-interaction kinds: the FP64 connection table of
// `conn_nodes` rows (negative: the batch has no connections) and, for FP32,
// the scratch of the starting prefix sum, 3 values per lane (FP64 with
// connections).
static size_t step_dyn_lds(bool f32, int waves, int conn_nodes)
{
    const size_t scan = (size_t)3 * 64 * waves;
    if (conn_nodes < 0) return f32 ? sizeof(float) * scan : 0;
    const size_t table = (size_t)6 * conn_nodes;
    return sizeof(double) * (f32 ? std::max(table, scan) : table);
}

template <typename T, int W>
static hipError_t launch_w(const DevBatch<T> &b, int n_sub, int grid, hipStream_t s)
{
    if (grid <= 0) grid = b.n_tiles;
    if (b.ext && (b.conn_idx || b.n_walls || b.cforce)) {
        // node interactions: the FP64 connection table (6 rows per connected
        // node), and for FP32 the scratch of the starting prefix sum (3 per lane)
        const size_t lds = step_dyn_lds(sizeof(T) == 4, W, b.conn_idx ? b.conn_nodes : -1);
        if ((b.n_walls || b.cforce) && b.conn_idx)
            hipLaunchKernelGGL((rod_step_kernel<T, W, 3>), dim3(grid), dim3(64 * W), lds, s, b, n_sub);
        else if (b.n_walls || b.cforce)
            hipLaunchKernelGGL((rod_step_kernel<T, W, 4>), dim3(grid), dim3(64 * W), lds, s, b, n_sub);
        else
            hipLaunchKernelGGL((rod_step_kernel<T, W, 2>), dim3(grid), dim3(64 * W), lds, s, b, n_sub);
    } else if (b.ext) {
        hipLaunchKernelGGL((rod_step_kernel<T, W, 1>), dim3(grid), dim3(64 * W), 0, s, b, n_sub);
    } else {
        hipLaunchKernelGGL((rod_step_kernel<T, W, 0>), dim3(grid), dim3(64 * W), 0, s, b, n_sub);
    }
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

hipError_t launch_set_step(int64_t *step, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, s, step, value);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *step, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step, n);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_energy_t(const DevBatch<T> &b, double *out, const int32_t *map, int n_map, hipStream_t s)
{
    const int bs = 64;
    const int rows = map ? n_map : b.n_rods;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL((rod_energy_kernel<T>), dim3((rows + bs - 1) / bs), dim3(bs), 0, s, b, out, map, n_map);
    return hipGetLastError();
}

hipError_t launch_energy(const DevBatch<double> &b, double *out, hipStream_t s)
{
    return launch_energy_t<double>(b, out, nullptr, 0, s);
}

hipError_t launch_energy(const DevBatch<float> &b, double *out, hipStream_t s, const int32_t *map, int n_map)
{
    return launch_energy_t<float>(b, out, map, n_map, s);
}

template <typename T, int W>
static int resident_w()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rod_step_kernel<T, W, 0>, 64 * W, 0) != hipSuccess)
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

template <typename T, int W, int KIND>
static size_t static_lds_w()
{
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void *>(rod_step_kernel<T, W, KIND>)) != hipSuccess) return 0;
    return a.sharedSizeBytes;
}

template <typename T, int KIND>
static size_t static_lds_t(int waves)
{
    switch (waves) {
    case 1: return static_lds_w<T, 1, KIND>();
    case 2: return static_lds_w<T, 2, KIND>();
    case 4: return static_lds_w<T, 4, KIND>();
    case 8: return static_lds_w<T, 8, KIND>();
    }
    return 0;
}

size_t step_lds_bytes(int precision_f32, int waves, int kind, int conn_nodes)
{
    size_t st = 0, dyn = 0;
    if (precision_f32) {
        st = kind == 4 ? static_lds_t<float, 4>(waves) : kind == 3 ? static_lds_t<float, 3>(waves)
           : kind == 2 ? static_lds_t<float, 2>(waves)
           : kind == 1 ? static_lds_t<float, 1>(waves) : static_lds_t<float, 0>(waves);
        if (kind >= 2) dyn = step_dyn_lds(true, waves, kind == 2 || conn_nodes > 0 ? conn_nodes : -1);
    } else {
        st = kind == 4 ? static_lds_t<double, 4>(waves) : kind == 3 ? static_lds_t<double, 3>(waves)
           : kind == 2 ? static_lds_t<double, 2>(waves)
           : kind == 1 ? static_lds_t<double, 1>(waves) : static_lds_t<double, 0>(waves);
        if (kind >= 2) dyn = step_dyn_lds(false, waves, conn_nodes);
    }
    return st + dyn;
}

}  // namespace rodk
