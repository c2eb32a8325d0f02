// contact_kernels.hip -- gfx950 kernels of rod-rod contact.
//
// Results, "Fibrous granular materials" (filaments in frictional contact;
// the paper names a GPU collision engine as future work and leaves the
// contact law to its supplement): every node is a sphere of its rod's
// radius; nodes of different rods that overlap push each other with the
// walls' penalty law (normal force delta (k - c v_n), regularised Coulomb
// friction).  One pass per step, before the step kernel's launch: bin the
// nodes (positions after the coming half drift) into a wrapped uniform grid
// with atomic counts, prefix-sum the counts, scatter the nodes into bucket
// order (each bucket sorted by node id), and let every node sum its contacts
// over the 27 buckets around it;
// the step kernel adds the forces at its kick.
#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace rodk {

namespace {

// Node id's rod, its position `drift` seconds ahead and its velocity (FP64
// state: lane node i at the slot, node n in the tail); false for padding slots
// and non-finite positions.
__device__ inline bool contact_node(const DevBatch<double> &B, const ContactGrid &, int64_t id, double drift,
                                    int &rod, double x[3], double v[3])
{
    const int64_t NS = B.n_slots;
    if (id < NS) {
        rod = B.slot_rod[id];
        if (rod < 0) return false;
        for (int a = 0; a < 3; ++a) {
            v[a] = B.state[(VX + a) * NS + id];
            x[a] = B.state[(RX + a) * NS + id] + drift * v[a];
        }
    } else {
        rod = (int)(id - NS);
        for (int a = 0; a < 3; ++a) {
            v[a] = B.tail[(TVX + a) * B.n_rods + rod];
            x[a] = B.tail[(TRX + a) * B.n_rods + rod] + drift * v[a];
        }
    }
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// FP32 batches hold edges and each rod's anchor: the positions come from
// contact_positions_kernel (already advanced by the drift), velocities from
// the state.
__device__ inline bool contact_node(const DevBatch<float> &B, const ContactGrid &G, int64_t id, double, int &rod,
                                    double x[3], double v[3])
{
    const int64_t NS = B.n_slots;
    if (id < NS) {
        rod = B.slot_rod[id];
        if (rod < 0) return false;
        for (int a = 0; a < 3; ++a) v[a] = (double)B.state[(VX + a) * NS + id];
    } else {
        rod = (int)(id - NS);
        for (int a = 0; a < 3; ++a) v[a] = (double)B.tail[(TVX + a) * B.n_rods + rod];
    }
    for (int a = 0; a < 3; ++a) x[a] = G.xabs[a * G.nn + id];
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// FP32 node positions for the grid: rod origin + anchor + the edges before
// the node, summed in FP64 and advanced by the drift.  One wave per rod: the
// lanes take 64 consecutive nodes at a time (coalesced loads and stores), an
// exclusive prefix sum of the FP32 edges across the lanes places them, and
// the chunk's total carries to the next 64.
__global__ __launch_bounds__(256) void contact_positions_kernel(const DevBatch<float> B, const ContactGrid G,
                                                                double drift)
{
    const int rod = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (rod >= B.n_rods) return;   // whole waves leave together
    const int64_t NS = B.n_slots, nn = G.nn, R = B.n_rods;
    const int n = B.rod_n[rod];
    const int64_t s0 = B.rod_slot[rod];
    double carry[3];
    for (int a = 0; a < 3; ++a) carry[a] = G.origin[a * R + rod] + (double)B.tail[(TRX + a) * R + rod];
    for (int base = 0; base <= n; base += 64) {
        const int j = base + lane;   // this lane's node; its edge j leads to node j + 1
        double incl[3];
        for (int a = 0; a < 3; ++a) incl[a] = j < n ? (double)B.state[(RX + a) * NS + s0 + j] : 0.0;
        for (int d = 1; d < 64; d <<= 1)
            for (int a = 0; a < 3; ++a) {
                const double up = __shfl_up(incl[a], d, 64);
                if (lane >= d) incl[a] += up;
            }
        double before[3];   // edges base .. j-1 (every lane takes part in the shuffle)
        for (int a = 0; a < 3; ++a) {
            const double up = __shfl_up(incl[a], 1, 64);
            before[a] = lane > 0 ? up : 0.0;
        }
        if (j <= n) {
            const int64_t id = j < n ? s0 + j : NS + rod;
            for (int a = 0; a < 3; ++a) {
                const double v = j < n ? (double)B.state[(VX + a) * NS + s0 + j] : (double)B.tail[(TVX + a) * R + rod];
                G.xabs[a * nn + id] = carry[a] + before[a] + drift * v;
            }
        }
        for (int a = 0; a < 3; ++a) carry[a] += __shfl(incl[a], 63, 64);
    }
}

__device__ inline int wrap_cell(int64_t c, int g)
{
    const int64_t m = c % g;
    return (int)(m < 0 ? m + g : m);
}

__device__ inline int64_t cell_of(double x, double org, double inv_cell)
{
    const double q = (x - org) * inv_cell;
    return (int64_t)floor(q < -1e15 ? -1e15 : (q > 1e15 ? 1e15 : q));   // finite x; keeps the cast defined
}

template <typename T>
__global__ void contact_bin_kernel(const DevBatch<T> B, const ContactGrid G, double drift)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn) return;
    int rod;
    double x[3], v[3];
    if (!contact_node(B, G, id, drift, rod, x, v)) {
        G.rank[id] = -1;
        return;
    }
    const int b = (wrap_cell(cell_of(x[2], G.org[2], G.inv_cell), G.gz) * G.gy
                   + wrap_cell(cell_of(x[1], G.org[1], G.inv_cell), G.gy)) * G.gx
                + wrap_cell(cell_of(x[0], G.org[0], G.inv_cell), G.gx);
    G.bucket[id] = b;
    G.rank[id] = atomicAdd(&G.count[b], 1);
}

// Exclusive prefix sum of the bucket counts: chunks of 1024 buckets (256
// threads x 4), then the chunk totals in one workgroup, then the offsets.
// The counts are cleared as they are read, ready for the next pass.
constexpr int SCAN_CHUNK = 1024;

__device__ inline int32_t block_exclusive(int32_t mine, int32_t *part, int n_threads, int32_t &total)
{
    const int t = threadIdx.x;
    part[t] = mine;
    __syncthreads();
    for (int off = 1; off < n_threads; off <<= 1) {
        const int32_t add = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    total = part[n_threads - 1];
    return part[t] - mine;
}

__global__ __launch_bounds__(256) void contact_scan_chunks(const ContactGrid G, int nb)
{
    __shared__ int32_t part[256];
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 4;
    int32_t c[4], sum = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k;
        c[k] = i < nb ? G.count[i] : 0;
        if (i < nb) G.count[i] = 0;
        sum += c[k];
    }
    int32_t total;
    int32_t run = block_exclusive(sum, part, 256, total);
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k;
        if (i < nb) G.start[i] = run;
        run += c[k];
    }
    if (threadIdx.x == 0) G.chunk[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void contact_scan_top(const ContactGrid G, int n_chunks, int nb)
{
    __shared__ int32_t part[1024];
    const int base = threadIdx.x * 4;
    int32_t c[4], sum = 0;
    for (int k = 0; k < 4; ++k) {
        c[k] = base + k < n_chunks ? G.chunk[base + k] : 0;
        sum += c[k];
    }
    int32_t total;
    int32_t run = block_exclusive(sum, part, 1024, total);
    for (int k = 0; k < 4; ++k) {
        if (base + k < n_chunks) G.chunk[base + k] = run;
        run += c[k];
    }
    if (threadIdx.x == 0) G.start[nb] = total;
}

__global__ __launch_bounds__(256) void contact_scan_add(const ContactGrid G, int nb)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 4;
    const int32_t off = G.chunk[blockIdx.x];
    for (int k = 0; k < 4; ++k)
        if (base + k < nb) G.start[base + k] += off;
}

template <typename T>
__global__ void contact_scatter_kernel(const DevBatch<T> B, const ContactGrid G, double drift)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn) return;
    const int32_t r = G.rank[id];
    if (r < 0) return;
    int rod;
    double x[3], v[3];
    contact_node(B, G, id, drift, rod, x, v);
    const int64_t p = G.start[G.bucket[id]] + r;
    G.spr[p] = make_double4(x[0], x[1], x[2], B.rod_rad[rod]);
    G.svr[p] = make_double4(v[0], v[1], v[2], (double)rod);
    G.sid[p] = (int32_t)id;
}

// The scatter leaves each bucket's nodes in the order their atomic ranks came
// out, which can differ from run to run; sorting every bucket by node id makes
// the order in which each node sums its contacts, and so the forces to the
// last bit, independent of the run.  Buckets hold a few nodes: insertion sort
// by the thread of the node that took rank 0 in the bucket (one per occupied
// bucket; threads run over node ids, far fewer than buckets).
__global__ void contact_sort_kernel(const ContactGrid G)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn || G.rank[id] != 0) return;
    const int b = G.bucket[id];
    const int32_t s = G.start[b], e = G.start[b + 1];
    for (int32_t i = s + 1; i < e; ++i) {
        const int32_t id = G.sid[i];
        if (G.sid[i - 1] < id) continue;
        const double4 a = G.spr[i], c = G.svr[i];
        int32_t j = i - 1;
        while (j >= s && G.sid[j] > id) {
            G.sid[j + 1] = G.sid[j];
            G.spr[j + 1] = G.spr[j];
            G.svr[j + 1] = G.svr[j];
            --j;
        }
        G.sid[j + 1] = id;
        G.spr[j + 1] = a;
        G.svr[j + 1] = c;
    }
}

// Each node sums its contacts with the nodes of other rods in the 27 buckets
// around it: the walls' law between two spheres.  Threads take the nodes in
// bucket order, so neighbouring threads read the same buckets and the sweep
// streams through the sorted records; a candidate costs one 32-byte load
// (position, radius), velocity and rod only for overlaps.  Results go to the
// node's id (padding ids keep the zeros set at creation).  (Renumbering the
// workgroups so that each XCD sweeps a contiguous eighth halved this kernel's
// HBM reads but made it slower on the fibre pile, so the plain order stays.)
template <typename T>
__global__ void contact_force_kernel(const DevBatch<T> B, const ContactGrid G, int nb)
{
    const int64_t p0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p0 >= G.start[nb]) return;
    const int64_t nn = G.nn;
    double f0 = 0, f1 = 0, f2 = 0, pot = 0;
    {
        const double4 me = G.spr[p0], mv = G.svr[p0];
        const int rod = (int)mv.w;
        const double x[3] = {me.x, me.y, me.z}, v[3] = {mv.x, mv.y, mv.z};
        const double ra = me.w;
        const double k = B.wall_k, c = B.wall_c, mu = B.wall_mu, vs = B.wall_vslip;
        const int64_t cx = cell_of(x[0], G.org[0], G.inv_cell), cy = cell_of(x[1], G.org[1], G.inv_cell),
                      cz = cell_of(x[2], G.org[2], G.inv_cell);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy) {
                const int row = (wrap_cell(cz + dz, G.gz) * G.gy + wrap_cell(cy + dy, G.gy)) * G.gx;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int b = row + wrap_cell(cx + dx, G.gx);
                    const int32_t p1 = G.start[b + 1];
                    for (int32_t p = G.start[b]; p < p1; ++p) {
                        const double4 q = G.spr[p];
                        const double e0 = x[0] - q.x, e1 = x[1] - q.y, e2 = x[2] - q.z;
                        const double d2 = e0 * e0 + e1 * e1 + e2 * e2, reach = ra + q.w;
                        if (!(d2 < reach * reach)) continue;
                        const double4 u = G.svr[p];
                        if ((int)u.w == rod) continue;
                        const double dist = sqrt(d2);
                        const double delta = reach - dist;
                        if (!(delta > 0.0)) continue;
                        pot += 0.25 * k * delta * delta;
                        if (!(dist > 0.0)) continue;   // coincident centres: no direction
                        const double n0 = e0 / dist, n1 = e1 / dist, n2 = e2 / dist;
                        const double r0 = v[0] - u.x, r1 = v[1] - u.y, r2 = v[2] - u.z;
                        const double vn = n0 * r0 + n1 * r1 + n2 * r2;
                        const double fn = delta * (k - c * vn);
                        if (!(fn > 0.0)) continue;
                        const double t0 = r0 - vn * n0, t1 = r1 - vn * n1, t2 = r2 - vn * n2;
                        const double sp = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
                        const double gf = mu * fn / (sp > vs ? sp : vs);
                        f0 += fn * n0 - gf * t0;
                        f1 += fn * n1 - gf * t1;
                        f2 += fn * n2 - gf * t2;
                    }
                }
            }
    }
    const int64_t id = G.sid[p0];
    G.force[id] = f0;
    G.force[nn + id] = f1;
    G.force[2 * nn + id] = f2;
    G.pot[id] = pot;
}

template <typename T>
hipError_t launch_contact_t(const DevBatch<T> &b, const ContactGrid &g, double drift, hipStream_t s)
{
    const int bs = 256;
    const int64_t nb64 = (int64_t)g.gx * g.gy * g.gz;
    if (g.nn <= 0) return hipSuccess;
    if (g.gx < 3 || g.gy < 3 || g.gz < 3 || nb64 > CONTACT_MAX_BUCKETS) return hipErrorInvalidValue;
    const int nb = (int)nb64;
    const int n_chunks = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const int gn = (int)((g.nn + bs - 1) / bs);
    if constexpr (sizeof(T) == 4) {
        if (!g.xabs || !g.origin) return hipErrorInvalidValue;
        hipLaunchKernelGGL(contact_positions_kernel, dim3((b.n_rods + 3) / 4), dim3(256), 0, s, b, g, drift);
    }
    hipLaunchKernelGGL((contact_bin_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift);
    hipLaunchKernelGGL(contact_scan_chunks, dim3(n_chunks), dim3(256), 0, s, g, nb);
    hipLaunchKernelGGL(contact_scan_top, dim3(1), dim3(1024), 0, s, g, n_chunks, nb);
    hipLaunchKernelGGL(contact_scan_add, dim3(n_chunks), dim3(256), 0, s, g, nb);
    hipLaunchKernelGGL((contact_scatter_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift);
    hipLaunchKernelGGL(contact_sort_kernel, dim3(gn), dim3(bs), 0, s, g);
    hipLaunchKernelGGL((contact_force_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, nb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_contact(const DevBatch<double> &b, const ContactGrid &g, double drift, hipStream_t s)
{
    return launch_contact_t<double>(b, g, drift, s);
}

hipError_t launch_contact(const DevBatch<float> &b, const ContactGrid &g, double drift, hipStream_t s)
{
    return launch_contact_t<float>(b, g, drift, s);
}

}  // namespace rodk
