// contact_kernels.hip -- gfx950 kernels of rod-rod contact.
//
// Results, "Fibrous granular materials" (filaments in frictional contact;
// the paper names a GPU collision engine as future work and leaves the
// contact law to its supplement).  Mode 1: every node is a sphere of its
// rod's radius; nodes of different rods that overlap push each other with the
// walls' penalty law (normal force delta (k - c v_n), regularised Coulomb
// friction).  Mode 2: every element is a capsule (its segment dilated by the
// radius); the same law acts between the closest points of two elements, of
// different rods or of one rod far enough apart along it, and each element's
// force goes to its two nodes.  One pass per step, before the step kernel's
// launch: bin the nodes or element midpoints (positions after the coming half
// drift) into a wrapped uniform grid with atomic counts, prefix-sum the
// counts, put the items into bucket order (each bucket sorted by id), and let
// every item sum its contacts over the 27 buckets around it; the step kernel
// adds the node forces at its kick.  Both modes can keep Verlet lists
// instead (a skin > 0): every node's list of partners (nodes of other rods
// within its radius plus the largest radius plus the skin at the build), or
// every element's (elements whose segments were within the two radii plus
// the skin), by increasing id.  A pass first sums each item's contacts over
// its list and checks how far every node has moved since the build; only when
// one has moved more than half the skin does the grid pass run, rebuilding
// the lists and summing every item's contacts again over its new list.  Both
// sums run over the same pairs (every pair that touches is listed) in the
// same order, so the forces depend neither on when the lists were built nor
// on the skin.
#include "rod.h"
#include "rod_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace rodk {

namespace {

// A position `drift` seconds ahead (one expression, so every caller rounds it
// alike).
__device__ inline double ahead(double r, double drift, double v) { return r + drift * v; }

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
            x[a] = ahead(B.state[(RX + a) * NS + id], drift, v[a]);
        }
    } else {
        rod = (int)(id - NS);
        for (int a = 0; a < 3; ++a) {
            v[a] = B.tail[(TVX + a) * B.n_rods + rod];
            x[a] = ahead(B.tail[(TRX + a) * B.n_rods + rod], drift, v[a]);
        }
    }
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// FP32 batches hold edges and each rod's anchor: the positions come from
// contact_positions_kernel (already advanced by the drift; in the Verlet
// records when the batch keeps lists), velocities from the state.
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
    if (G.rec) {
        const double4 r = G.rec[2 * id];
        x[0] = r.x;
        x[1] = r.y;
        x[2] = r.z;
    } else {
        for (int a = 0; a < 3; ++a) x[a] = G.xabs[a * G.nid + id];
    }
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// FP32 node positions for the grid: rod origin + anchor + the edges before
// the node, summed in FP64 and advanced by the drift.  One wave per rod: the
// lanes take 64 consecutive nodes at a time (coalesced loads and stores), an
// exclusive prefix sum of the FP32 edges across the lanes places them, and
// the chunk's total carries to the next 64.  With Verlet lists the positions
// go into the nodes' records instead, with the move check of the pack kernel
// below.
__global__ __launch_bounds__(256) void contact_positions_kernel(const DevBatch<float> B, const ContactGrid G,
                                                                double drift)
{
    const int rod = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (rod >= B.n_rods) return;   // whole waves leave together
    const int64_t NS = B.n_slots, nn = G.nid, R = B.n_rods;
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
        int moved = 0;
        if (j <= n) {
            const int64_t id = j < n ? s0 + j : NS + rod;
            double x[3], v[3];
            for (int a = 0; a < 3; ++a) {
                v[a] = j < n ? (double)B.state[(VX + a) * NS + s0 + j] : (double)B.tail[(TVX + a) * R + rod];
                x[a] = carry[a] + before[a] + drift * v[a];
            }
            if (G.rec) {
                G.rec[2 * id] = make_double4(x[0], x[1], x[2], B.rod_rad[rod]);
                G.rec[2 * id + 1] = make_double4(v[0], v[1], v[2], (double)rod);
                if (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2])) {
                    const double h = 0.5 * G.skin;
                    const double e0 = x[0] - G.xb[id], e1 = x[1] - G.xb[nn + id], e2 = x[2] - G.xb[2 * nn + id];
                    moved = !(e0 * e0 + e1 * e1 + e2 * e2 <= h * h);
                } else {
                    G.xb[id] = NAN;   // a node that turns finite again (a new state) forces a build
                }
            } else {
                for (int a = 0; a < 3; ++a) G.xabs[a * nn + id] = x[a];
            }
        }
        if (__any(moved) && lane == 0) atomicOr(&G.vflag[VF_REQUEST], 1);
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

// With Verlet lists a kernel of the pass runs only when a flag set by the
// check before it says so (the flag's value, set or clear, is the same for
// every thread of the launch); without (p NULL) it always runs.
struct Gate {
    const int32_t *p = nullptr;
    int want = 1;
    __device__ bool skip() const { return p && ((*p != 0) != (want != 0)); }
};

template <typename T>
__global__ void contact_bin_kernel(const DevBatch<T> B, const ContactGrid G, double drift, Gate gate)
{
    if (gate.skip()) return;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn) return;
    if (G.need) G.need[id] = 0;   // the build marks the records its lists use
    int rod;
    double x[3], v[3];
    if (!contact_node(B, G, id, drift, rod, x, v)) {
        G.rank[id] = -1;
        if (G.lcount) G.lcount[id] = 0;   // not binned: no partners until the next build
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

__global__ __launch_bounds__(256) void contact_scan_chunks(const ContactGrid G, int nb, Gate gate)
{
    if (gate.skip()) return;
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

__global__ __launch_bounds__(1024) void contact_scan_top(const ContactGrid G, int n_chunks, int nb, Gate gate)
{
    if (gate.skip()) return;
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

__global__ __launch_bounds__(256) void contact_scan_add(const ContactGrid G, int nb, Gate gate)
{
    if (gate.skip()) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 4;
    const int32_t off = G.chunk[blockIdx.x];
    for (int k = 0; k < 4; ++k)
        if (base + k < nb) G.start[base + k] += off;
}

template <typename T>
__global__ void contact_scatter_kernel(const DevBatch<T> B, const ContactGrid G, double drift, Gate gate)
{
    if (gate.skip()) return;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn) return;
    const int32_t r = G.rank[id];
    if (r < 0) return;
    int rod;
    double x[3], v[3];
    contact_node(B, G, id, drift, rod, x, v);
    const int64_t p = G.start[G.bucket[id]] + r;
    G.spr[p] = make_double4(x[0], x[1], x[2], (double)rod);
    G.svr[p] = make_double4(v[0], v[1], v[2], B.rod_rad[rod]);
    G.sid[p] = (int32_t)id;
}

// The scatter leaves each bucket's nodes in the order their atomic ranks came
// out, which can differ from run to run; sorting every bucket by node id makes
// the order in which each node sums its contacts, and so the forces to the
// last bit, independent of the run.  Buckets hold a few nodes: insertion sort
// by the thread of the node that took rank 0 in the bucket (one per occupied
// bucket; threads run over node ids, far fewer than buckets).
__global__ void contact_sort_kernel(const ContactGrid G, Gate gate)
{
    if (gate.skip()) return;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn || G.rank[id] != 0) return;
    const int b = G.bucket[id];
    const int32_t s = G.start[b], e = G.start[b + 1];
    for (int32_t i = s + 1; i < e; ++i) {
        const int32_t key = G.sid[i];
        if (G.sid[i - 1] < key) continue;
        const double4 a = G.spr[i], c = G.svr[i];
        int32_t j = i - 1;
        while (j >= s && G.sid[j] > key) {
            G.sid[j + 1] = G.sid[j];
            G.spr[j + 1] = G.spr[j];
            G.svr[j + 1] = G.svr[j];
            --j;
        }
        G.sid[j + 1] = key;
        G.spr[j + 1] = a;
        G.svr[j + 1] = c;
    }
}

// Force passes: workgroups of CF_BLOCK lanes, one item per lane; a lane
// screens its candidates CF_GROUP at a time (their records loaded together,
// the test without branches; the record arrays hold CONTACT_PAD entries past
// the last item, so a group may read past a range's end and mask what it
// read) and queues the survivors' sorted positions in LDS, CF_QUEUE at most.
// A lane screens until its queue is nearly full or its sweep ends; then the
// wave evaluates its queues together, each lane taking its survivors in the
// order it queued them (the order of the sweep, so the sums are those of a
// single pass), and lanes with candidates left go on.
constexpr int CF_BLOCK = 256;
constexpr int CF_QUEUE = 32;   // survivors a lane holds (LDS: 32 KB per workgroup)
constexpr int CF_GROUP = 4;
static_assert(CF_GROUP <= CONTACT_PAD, "a group may read up to CF_GROUP - 1 records past the last item");

// A lane's sweep over the sorted positions of the 27 buckets around cell
// (cx, cy, cz) in bucket order: 27 ranges, or 9 rows of three contiguous x
// buckets where the row does not wrap there.  next() moves p..pe to the next
// non-empty range and returns false at the end.  The bounds of the range
// after the current one are loaded ahead (np, npe), so their latency overlaps
// the screening of the current range.
struct Sweep {
    int64_t cx, cy, cz;
    int wx, ri;
    bool run;
    int32_t p, pe, np, npe;   // np = -1: no range left
    __device__ Sweep(const ContactGrid &G, int64_t x, int64_t y, int64_t z)
        : cx(x), cy(y), cz(z), wx(wrap_cell(x, G.gx)), ri(0), run(false), p(0), pe(0), np(-1), npe(0)
    {
        run = wx >= 1 && wx + 1 < G.gx;
        fetch(G);
    }
    // bounds of range ri into np, npe
    __device__ void fetch(const ContactGrid &G)
    {
        if (ri >= 27) {
            np = -1;
            return;
        }
        const int r = ri / 3;
        const int row = (wrap_cell(cz + r / 3 - 1, G.gz) * G.gy + wrap_cell(cy + r % 3 - 1, G.gy)) * G.gx;
        const int b0 = run ? row + wx - 1 : row + wrap_cell(cx + ri % 3 - 1, G.gx);
        const int b1 = run ? row + wx + 2 : b0 + 1;
        np = G.start[b0];
        npe = G.start[b1];
        ri += run ? 3 : 1;
    }
    __device__ bool next(const ContactGrid &G)
    {
        for (;;) {
            if (np < 0) return false;
            p = np;
            pe = npe;
            fetch(G);
            if (p < pe) return true;
        }
    }
};

// Workgroup index in a renumbering that gives each XCD a contiguous run of
// workgroups (the hardware deals them out to the 8 XCDs in turn), so each
// XCD's L2 holds the records of one region of the sorted order.
__device__ inline int64_t xcd_contiguous_block()
{
    const int nb = gridDim.x, x = blockIdx.x % 8, i = blockIdx.x / 8;
    const int q = nb / 8, r = nb % 8;
    return (int64_t)x * q + (x < r ? x : r) + i;
}

// The walls' law between two spheres: node a at x (velocity v, radius ra)
// against a partner at q (velocity u, radius rb); adds a's force to f and
// a's share of the pair's potential (half) to pot.
__device__ __attribute__((always_inline)) inline void sphere_pair(const double x[3], const double v[3], double ra, const double4 &q, const double4 &u,
                                   double rb, double k, double c, double mu, double vs, double f[3], double &pot)
{
    const double e0 = x[0] - q.x, e1 = x[1] - q.y, e2 = x[2] - q.z;
    const double d2 = e0 * e0 + e1 * e1 + e2 * e2, reach = ra + rb;
    if (!(d2 < reach * reach)) return;
    const double dist = sqrt(d2);
    const double delta = reach - dist;
    if (!(delta > 0.0)) return;
    pot += 0.25 * k * delta * delta;
    if (!(dist > 0.0)) return;   // coincident centres: no direction
    const double n0 = e0 / dist, n1 = e1 / dist, n2 = e2 / dist;
    const double r0 = v[0] - u.x, r1 = v[1] - u.y, r2 = v[2] - u.z;
    const double vn = n0 * r0 + n1 * r1 + n2 * r2;
    const double fn = delta * (k - c * vn);
    if (!(fn > 0.0)) return;
    const double t0 = r0 - vn * n0, t1 = r1 - vn * n1, t2 = r2 - vn * n2;
    const double sp = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    const double gf = mu * fn / (sp > vs ? sp : vs);
    f[0] += fn * n0 - gf * t0;
    f[1] += fn * n1 - gf * t1;
    f[2] += fn * n2 - gf * t2;
}

// Verlet lists: every node's record for the pass, two double4 per id:
// (position after the drift, radius) and (velocity, rod; -1 for padding).
// A node that is not finite fails every pair's distance test.
__device__ __attribute__((always_inline)) inline void node_record(const ContactGrid &G, int64_t p, double4 &y, double4 &u)
{
    y = G.rec[2 * p];
    u = G.rec[2 * p + 1];
}

// Up to four listed pairs of a node (entries e[0..m-1]; the rest are ignored
// but must name valid nodes): the partners' records all load before the
// pairs are evaluated, in entry order.
template <typename T>
__device__ __attribute__((always_inline)) inline void listed_pairs4(const DevBatch<T> &B, const ContactGrid &G, const int32_t e[4], int m,
                                     const double x[3], const double v[3], double ra, double f[3], double &pot)
{
    const double k = B.wall_k, c = B.wall_c, mu = B.wall_mu, vs = B.wall_vslip;
    double4 y[4], u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) node_record(G, e[q], y[q], u[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < m) sphere_pair(x, v, ra, y[q], u[q], y[q].w, k, c, mu, vs, f, pot);
}

// A node's contacts over its Verlet list entries j0 .. n-1, in list
// (increasing id) order, four entries at a time (entries past the end repeat
// the last one and are not evaluated).
template <typename T>
__device__ __attribute__((always_inline)) inline void list_contacts(const DevBatch<T> &B, const ContactGrid &G, int64_t id, int j0, int n,
                                     const double x[3], const double v[3], double ra, double f[3], double &pot)
{
    for (; j0 < n; j0 += 4) {
        int32_t e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = G.lid[min(j0 + q, n - 1) * G.nid + id];
        listed_pairs4(B, G, e, n - j0, x, v, ra, f, pot);
    }
}

// The same sum, each partner read as contact_node gives it (the values the
// records hold), for the pass that builds the lists: in FP64 batches records
// are written only for the nodes the previous lists used.  A partner that is not finite
// adds nothing, as its record's failed distance test does.
template <typename T>
__device__ __attribute__((always_inline)) inline void list_contacts_state(const DevBatch<T> &B, const ContactGrid &G, int64_t id, int n,
                                           double drift, const double x[3], const double v[3], double ra,
                                           double f[3], double &pot)
{
    const double k = B.wall_k, c = B.wall_c, mu = B.wall_mu, vs = B.wall_vslip;
    for (int j = 0; j < n; ++j) {
        int rb;
        double y[3], u[3];
        if (!contact_node(B, G, G.lid[j * G.nid + id], drift, rb, y, u)) continue;
        sphere_pair(x, v, ra, make_double4(y[0], y[1], y[2], 0.0), make_double4(u[0], u[1], u[2], 0.0),
                    B.rod_rad[rb], k, c, mu, vs, f, pot);
    }
}

// Each node sums its contacts with the nodes of other rods in the 27 buckets
// around it: the walls' law between two spheres.  Threads take the nodes in
// bucket order, so neighbouring threads read the same buckets.  The screen
// keeps candidates of other rods closer than the node's radius plus the
// largest radius (a bound on the exact test, widened by 1e-9 relative so that
// rounding cannot drop a pair the exact test takes); the evaluation repeats
// the exact test with the partner's radius and applies the law.  Results go
// to the node's id (padding ids keep the zeros set at creation).
// LIST (the pass that rebuilds the Verlet lists): the screen's bound grows by
// the skin and every survivor's id joins the node's list, which is then
// sorted by id; the node's contacts are summed over the new list, or, when
// it overflowed, in the sweep's order (the evaluation above, run on the same
// survivors), and the next pass is asked to build again.
template <typename T, bool LIST>
__global__ __launch_bounds__(CF_BLOCK) void contact_force_kernel(const DevBatch<T> B, const ContactGrid G, int nb,
                                                                 double drift, Gate gate)
{
    if (gate.skip()) return;
    __shared__ int32_t queue[CF_QUEUE * CF_BLOCK];
    int32_t *const mine = queue + threadIdx.x;   // entry j at mine[j * CF_BLOCK]
    const int64_t p0 = xcd_contiguous_block() * CF_BLOCK + threadIdx.x;
    // no early exit: every lane reaches the wave-wide evaluations
    const bool live = p0 < G.start[nb];
    const int64_t pm = live ? p0 : 0;
    const double4 me = G.spr[pm], mv = G.svr[pm];
    const int rod = (int)me.w;
    const double x[3] = {me.x, me.y, me.z}, v[3] = {mv.x, mv.y, mv.z};
    const double ra = mv.w;
    const double rs = LIST ? ra + G.rmax + G.skin : ra + G.rmax, rs2 = rs * rs * (1.0 + 1e-9);
    const double k = B.wall_k, c = B.wall_c, mu = B.wall_mu, vs = B.wall_vslip;
    double f[3] = {0.0, 0.0, 0.0}, pot = 0;
    int nq = 0;
    const int64_t id = live ? G.sid[p0] : 0, NI = G.nid;
    int n_list = 0;

    Sweep sw(G, cell_of(x[0], G.org[0], G.inv_cell), cell_of(x[1], G.org[1], G.inv_cell),
             cell_of(x[2], G.org[2], G.inv_cell));
    bool done = !live || !sw.next(G);
    for (;;) {
        while (!done && nq <= CF_QUEUE - CF_GROUP) {
            const double4 *const q = G.spr + sw.p;
            double4 r[CF_GROUP];
#pragma unroll
            for (int u = 0; u < CF_GROUP; ++u) r[u] = q[u];
#pragma unroll
            for (int u = 0; u < CF_GROUP; ++u) {
                const double e0 = x[0] - r[u].x, e1 = x[1] - r[u].y, e2 = x[2] - r[u].z;
                const bool ok = (sw.p + u < sw.pe) & (e0 * e0 + e1 * e1 + e2 * e2 < rs2) & ((int)r[u].w != rod);
                mine[nq * CF_BLOCK] = sw.p + u;   // nq < CF_QUEUE: a free slot, kept only if it passed
                nq += (int)ok;
            }
            sw.p += CF_GROUP;
            if (sw.p >= sw.pe) done = !sw.next(G);
        }
        for (int j = 0; j < nq; ++j) {
            const int32_t p = mine[j * CF_BLOCK];
            const double4 u = G.svr[p];
            sphere_pair(x, v, ra, G.spr[p], u, u.w, k, c, mu, vs, f, pot);
            if constexpr (LIST) {
                if (n_list < CONTACT_LIST_CAP) G.lid[n_list * NI + id] = G.sid[p];
                ++n_list;
            }
        }
        nq = 0;
        if (!__any(!done)) break;
    }
    if constexpr (LIST) {
        int most = n_list;   // the wave's longest list, one atomic per wave
        for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o, 64));
        if ((threadIdx.x & 63) == 0 && most > 0) atomicMax(&G.vflag[VF_MOST], most);
        if (!live) return;
        for (int a = 0; a < 3; ++a) G.xb[a * NI + id] = x[a];
        G.lcount[id] = n_list;
        if (n_list > CONTACT_LIST_CAP) {
            atomicOr(&G.vflag[VF_OVERFLOW], 1);   // forces of the sweep's order; the next pass builds again
        } else {
            int32_t *const L = G.lid + id;   // insertion sort by id (the sweep left it sorted within buckets)
            for (int i = 1; i < n_list; ++i) {
                const int32_t key = L[i * NI];
                int j = i - 1;
                while (j >= 0 && L[j * NI] > key) {
                    L[(j + 1) * NI] = L[j * NI];
                    --j;
                }
                L[(j + 1) * NI] = key;
            }
            f[0] = f[1] = f[2] = pot = 0.0;
            list_contacts_state(B, G, id, n_list, drift, x, v, ra, f, pot);
            if (G.need && n_list > 0) {   // the records the list pass will read
                G.need[id] = 1;
                for (int j = 0; j < n_list; ++j) G.need[L[j * NI]] = 1;
            }
        }
    }
    if (!live) return;
    G.force[id] = f[0];
    G.force[NI + id] = f[1];
    G.force[2 * NI + id] = f[2];
    G.pot[id] = pot;
}

// A node's position `drift` ahead and velocity, as contact_node gives them,
// without its branches: slot and tail arrays keep position and velocity at
// the same field offsets.
static_assert((int)RX == (int)TRX && (int)VX == (int)TVX, "slot and tail fields share offsets");

__device__ inline void node_state(const DevBatch<double> &B, const ContactGrid &, int64_t p, double drift,
                                  double x[3], double v[3])
{
    const int64_t NS = B.n_slots;
    const bool slot = p < NS;
    const double *const src = slot ? B.state + p : B.tail + (p - NS);
    const int64_t st = slot ? NS : B.n_rods;
    for (int a = 0; a < 3; ++a) v[a] = src[(VX + a) * st];
    for (int a = 0; a < 3; ++a) x[a] = ahead(src[(RX + a) * st], drift, v[a]);
}

__device__ inline void node_state(const DevBatch<float> &B, const ContactGrid &G, int64_t p, double, double x[3],
                                  double v[3])
{
    const int64_t NS = B.n_slots;
    const bool slot = p < NS;
    const float *const src = slot ? B.state + p : B.tail + (p - NS);
    const int64_t st = slot ? NS : B.n_rods;
    for (int a = 0; a < 3; ++a) v[a] = (double)src[(VX + a) * st];
    for (int a = 0; a < 3; ++a) x[a] = G.xabs[a * G.nid + p];
}

// Verlet lists, first kernel of every pass (FP64 batches; FP32 batches do
// this in the positions kernel): the record (above) of every node the last
// build's lists use, and a request for a build when any node has moved more
// than half the skin from its position at the build (a NaN position there
// counts as moved).  Without a build no pair missing from the lists can
// touch: the pair was at least its radii plus the skin apart at the build (up
// to the 1e-9 widening) and each node has moved at most half the skin since.
template <typename T>
__global__ __launch_bounds__(256) void verlet_pack_kernel(const DevBatch<T> B, const ContactGrid G, double drift)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, NI = G.nid, NS = B.n_slots;
    // every load goes out at once (ids past the end read the last id's)
    const int64_t ic = id < NI ? id : NI - 1;
    const int rod = ic < NS ? B.slot_rod[ic] : (int)(ic - NS);
    double x[3], v[3];
    node_state(B, G, ic, drift, x, v);
    const double b0 = G.xb[ic], b1 = G.xb[NI + ic], b2 = G.xb[2 * NI + ic];
    const double rad = B.rod_rad[rod < 0 ? 0 : rod];
    const bool need = G.need[ic] != 0;
    const bool live = id < NI && rod >= 0;
    const bool ok = live && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
    const double h = 0.5 * G.skin, e0 = x[0] - b0, e1 = x[1] - b1, e2 = x[2] - b2;
    const int moved = ok && !(e0 * e0 + e1 * e1 + e2 * e2 <= h * h);
    if (__any(moved) && (threadIdx.x & 63) == 0) atomicOr(&G.vflag[VF_REQUEST], 1);
    if (!live) return;
    if (need) {   // a node with partners, or some node's partner, at the last build
        G.rec[2 * id] = make_double4(x[0], x[1], x[2], rad);
        G.rec[2 * id + 1] = make_double4(v[0], v[1], v[2], (double)rod);
    }
    if (!ok) G.xb[id] = NAN;   // a node that turns finite again (a new state) forces a build
}

// Verlet lists, every pass: each node with partners sums its contacts over
// its list from the records.  A node without partners (padding ids too)
// reads and writes nothing: its force and potential are the zeros the last
// build wrote (or creation's).  With a build in this pass the forces
// computed here are replaced.
template <typename T>
__global__ __launch_bounds__(256) void verlet_force_kernel(const DevBatch<T> B, const ContactGrid G)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, NI = G.nid;
    if (id >= NI) return;
    const int n = min(G.lcount[id], CONTACT_LIST_CAP);   // larger only after an overflow, when a build follows
    if (n == 0) return;
    double4 y, u;
    node_record(G, id, y, u);
    double f[3] = {0.0, 0.0, 0.0}, pot = 0;
    const double x[3] = {y.x, y.y, y.z}, v[3] = {u.x, u.y, u.z};
    list_contacts(B, G, id, 0, n, x, v, y.w, f, pot);
    G.force[id] = f[0];
    G.force[NI + id] = f[1];
    G.force[2 * NI + id] = f[2];
    G.pot[id] = pot;
}

// Verlet lists, the end of a pass (after the step kernel, in place of its
// step-counter advance): counts the pass and its build, carries an overflow
// of this pass's build into the next pass's request, and clears the flags.
__global__ void verlet_finish_kernel(int32_t *vflag, int64_t *step, int64_t n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (step) *step += n;
    const int req = vflag[VF_REQUEST], ovf = vflag[VF_OVERFLOW];
    vflag[VF_PASSES] += 1;
    vflag[VF_BUILDS] += req != 0;
    vflag[VF_FALLBACKS] += ovf != 0;
    vflag[VF_REQUEST] = ovf;
    vflag[VF_OVERFLOW] = 0;
}

// ---------------------------------------------------------------- capsules
// Mode 2: every element is a capsule, the segment between its nodes A (node
// i) and B (node i + 1) dilated by the rod's radius.  Elements are binned by
// their midpoints in cells of the longest element the grid allows for plus
// twice the largest radius, so the midpoints of two touching elements are at
// most one cell apart per axis.

// Each binned item's id to its place: the bucket's start plus its rank.
__global__ void contact_scatter_ids(const ContactGrid G, Gate gate)
{
    if (gate.skip()) return;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn) return;
    const int32_t r = G.rank[id];
    if (r < 0) return;
    G.sid[G.start[G.bucket[id]] + r] = (int32_t)id;
}

// As contact_sort_kernel, for the ids alone: the segment records (128 bytes
// each) are written afterwards, in sorted order, by seg_fill_kernel.
__global__ void sort_ids_kernel(const ContactGrid G, Gate gate)
{
    if (gate.skip()) return;
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nn || G.rank[id] != 0) return;
    const int b = G.bucket[id];
    const int32_t s = G.start[b], e = G.start[b + 1];
    for (int32_t i = s + 1; i < e; ++i) {
        const int32_t key = G.sid[i];
        int32_t j = i - 1;
        while (j >= s && G.sid[j] > key) {
            G.sid[j + 1] = G.sid[j];
            --j;
        }
        G.sid[j + 1] = key;
    }
}

// FP32 screening record of an element, two float4: the centre of its
// capsule's axis-aligned bounding box relative to the grid origin and the half
// extents, then its rod and element index (as bits).
__device__ inline void cull_record(const double a[3], const double b[3], double r, int rod, int elem,
                                   const ContactGrid &G, float4 &c0, float4 &c1)
{
    double c[3], e[3];
    for (int k = 0; k < 3; ++k) {
        const double lo = fmin(a[k], b[k]) - r, hi = fmax(a[k], b[k]) + r;
        c[k] = 0.5 * (lo + hi) - G.org[k];
        e[k] = 0.5 * (hi - lo);
    }
    c0 = make_float4((float)c[0], (float)c[1], (float)c[2], (float)e[0]);
    c1 = make_float4((float)e[1], (float)e[2], __int_as_float(rod), __int_as_float(elem));
}

// Screening tolerance of a box test in FP32.  Two capsules in contact have
// boxes that overlap in exact arithmetic: per axis, the centres are closer
// than the sum of the half extents, itself at most a cell or so.  Rounding
// each centre (relative to the origin) and half extent to FP32 moves the two
// sides of the test by at most 2^-24 times the centres' magnitudes plus the
// extents, below 2^-23 (|c|_1 + 2 cell) for the element's own centre c, and
// the FP32 test itself adds a unit or two of 2^-24 of the same.  The margin
// 1e-6 (|c|_1 + 4 cell) > 2^-20 (|c|_1 + 4 cell) covers this eight times
// over, so the screen drops only pairs that cannot touch.
__device__ inline float cull_margin(const float4 &c, float cell)
{
    return 1e-6f * (fabsf(c.x) + fabsf(c.y) + fabsf(c.z) + 4.0f * cell);
}

// Element (slot) s: endpoints and velocities `drift` seconds ahead; false for
// padding slots and non-finite positions.
template <typename T>
__device__ inline bool contact_segment(const DevBatch<T> &B, const ContactGrid &G, int64_t s, double drift, int &rod,
                                       int &elem, double a[3], double b[3], double va[3], double vb[3])
{
    rod = B.slot_rod[s];
    if (rod < 0) return false;
    elem = B.slot_idx[s];
    const int64_t idb = elem + 1 < B.rod_n[rod] ? s + 1 : B.n_slots + rod;
    int r2;
    const bool oka = contact_node(B, G, s, drift, r2, a, va);
    const bool okb = contact_node(B, G, idb, drift, r2, b, vb);
    return oka && okb;
}

// Closest points p0 + s (p1 - p0), q0 + t (q1 - q0) of two segments of
// positive length, s, t in [0, 1]: the convex quadratic's stationary s,
// clamped; the best t for it, clamped; s again for a clamped t; s from 0 for
// parallel segments.
__device__ __attribute__((always_inline)) inline void closest_params(const double p0[3], const double p1[3], const double q0[3], const double q1[3],
                                      double &s, double &t)
{
    const double d1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double d2[3] = {q1[0] - q0[0], q1[1] - q0[1], q1[2] - q0[2]};
    const double r[3] = {p0[0] - q0[0], p0[1] - q0[1], p0[2] - q0[2]};
    const double a = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
    const double e = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
    const double b = d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2];
    const double c = d1[0] * r[0] + d1[1] * r[1] + d1[2] * r[2];
    const double f = d2[0] * r[0] + d2[1] * r[1] + d2[2] * r[2];
    const double den = a * e - b * b;
    double ss = 0.0;
    if (den > 1e-12 * a * e) ss = fmin(fmax((b * f - c * e) / den, 0.0), 1.0);
    double tt = (b * ss + f) / e;
    if (tt < 0.0) {
        tt = 0.0;
        ss = fmin(fmax(-c / a, 0.0), 1.0);
    } else if (tt > 1.0) {
        tt = 1.0;
        ss = fmin(fmax((b - c) / a, 0.0), 1.0);
    }
    s = ss;
    t = tt;
}

template <typename T>
__global__ void seg_bin_kernel(const DevBatch<T> B, const ContactGrid G, double drift, Gate gate)
{
    if (gate.skip()) return;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= G.nn) return;
    int rod, elem;
    double a[3], b[3], va[3], vb[3];
    const bool ok = contact_segment(B, G, s, drift, rod, elem, a, b, va, vb);
    if (G.lcount && rod >= 0) {
        // Verlet lists: the build's positions of the element's node A, and of
        // the rod's last node after its last element (NaN where not finite)
        const int64_t NI = G.nid;
        for (int k = 0; k < 3; ++k) G.xb[k * NI + s] = a[k];
        if (elem + 1 == B.rod_n[rod])
            for (int k = 0; k < 3; ++k) G.xb[k * NI + B.n_slots + rod] = b[k];
        if (!ok) G.lcount[s] = 0;   // not binned: no partners until the next build
    }
    if (!ok) {
        // out of the grid this pass: its nodes take no shares from it
        G.rank[s] = -1;
        for (int k = 0; k < 6; ++k) G.fseg[k * G.nn + s] = 0.0;
        G.pot[s] = 0.0;
        return;
    }
    // longer than the grid's cells allow for: contacts of this element may be missed
    const double l2 = (b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]);
    if (l2 > G.cell_len * G.cell_len) atomicOr(&B.nonfinite[rod], ROD_FLAG_STRETCHED);
    const int bk = (wrap_cell(cell_of(0.5 * (a[2] + b[2]), G.org[2], G.inv_cell), G.gz) * G.gy
                    + wrap_cell(cell_of(0.5 * (a[1] + b[1]), G.org[1], G.inv_cell), G.gy)) * G.gx
                 + wrap_cell(cell_of(0.5 * (a[0] + b[0]), G.org[0], G.inv_cell), G.gx);
    G.bucket[s] = bk;
    G.rank[s] = atomicAdd(&G.count[bk], 1);
}

// Segment records in sorted order: (A, radius), (B, rod), (v_A, element),
// v_B, and the screening record.
template <typename T>
__global__ void seg_fill_kernel(const DevBatch<T> B, const ContactGrid G, double drift, int nb, Gate gate)
{
    if (gate.skip()) return;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= G.start[nb]) return;
    const int64_t s = G.sid[p];
    int rod, elem;
    double a[3], b[3], va[3], vb[3];
    contact_segment(B, G, s, drift, rod, elem, a, b, va, vb);
    const double r = B.rod_rad[rod];
    G.sca[p] = make_double4(a[0], a[1], a[2], r);
    G.scb[p] = make_double4(b[0], b[1], b[2], (double)rod);
    G.sva[p] = make_double4(va[0], va[1], va[2], (double)elem);
    G.svb[p] = make_double4(vb[0], vb[1], vb[2], 0.0);
    cull_record(a, b, r, rod, elem, G, G.cull[2 * p], G.cull[2 * p + 1]);
}

// One capsule pair, seen from element e (records ua = (A, radius), ub = (B,
// rod), uva = (v_A, element), uvb = v_B) against element q (qa, qb, qva, qvb):
// the closest points and the force in one fixed order (the element first in
// (rod, element) order takes the part of u), e taking the exact negative when
// it is the second, so the two feel opposite forces to the last bit.  The
// force goes to e's nodes as (1 - s) and s; a quarter of k delta^2 per
// ordered pair is e's potential share.  Returns the closest points' distance.
__device__ __attribute__((always_inline)) inline double capsule_pair(const double4 &ua, const double4 &ub, const double4 &uva, const double4 &uvb,
                                      const double4 &qa, const double4 &qb, const double4 &qva, const double4 &qvb,
                                      double k, double c, double mu, double vs, double fa[3], double fb[3],
                                      double &pot)
{
    const int rod = (int)ub.w, elem = (int)uva.w;
    const int qrod = (int)qb.w, qelem = (int)qva.w;
    const double ra = ua.w;
    const bool first = rod < qrod || (rod == qrod && elem < qelem);
    // u: the pair's first element, w: the other
    const double u0[3] = {first ? ua.x : qa.x, first ? ua.y : qa.y, first ? ua.z : qa.z};
    const double u1[3] = {first ? ub.x : qb.x, first ? ub.y : qb.y, first ? ub.z : qb.z};
    const double w0[3] = {first ? qa.x : ua.x, first ? qa.y : ua.y, first ? qa.z : ua.z};
    const double w1[3] = {first ? qb.x : ub.x, first ? qb.y : ub.y, first ? qb.z : ub.z};
    // the velocities picked component by component (a select of whole
    // records would go through memory)
    const double vu0[3] = {first ? uva.x : qva.x, first ? uva.y : qva.y, first ? uva.z : qva.z};
    const double vu1[3] = {first ? uvb.x : qvb.x, first ? uvb.y : qvb.y, first ? uvb.z : qvb.z};
    const double vw0[3] = {first ? qva.x : uva.x, first ? qva.y : uva.y, first ? qva.z : uva.z};
    const double vw1[3] = {first ? qvb.x : uvb.x, first ? qvb.y : uvb.y, first ? qvb.z : uvb.z};
    const double ru = first ? ra : qa.w, rw = first ? qa.w : ra;
    double su, sw;
    closest_params(u0, u1, w0, w1, su, sw);
    const double pu[3] = {u0[0] + su * (u1[0] - u0[0]), u0[1] + su * (u1[1] - u0[1]), u0[2] + su * (u1[2] - u0[2])};
    const double pw[3] = {w0[0] + sw * (w1[0] - w0[0]), w0[1] + sw * (w1[1] - w0[1]), w0[2] + sw * (w1[2] - w0[2])};
    const double e0 = pu[0] - pw[0], e1 = pu[1] - pw[1], e2 = pu[2] - pw[2];
    const double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    const double delta = ru + rw - dist;
    if (!(delta > 0.0)) return dist;
    pot += 0.25 * k * delta * delta;
    if (!(dist > 0.0)) return dist;   // the segments cross: no direction
    const double n0 = e0 / dist, n1 = e1 / dist, n2 = e2 / dist;
    const double r0 = ((1.0 - su) * vu0[0] + su * vu1[0]) - ((1.0 - sw) * vw0[0] + sw * vw1[0]);
    const double r1 = ((1.0 - su) * vu0[1] + su * vu1[1]) - ((1.0 - sw) * vw0[1] + sw * vw1[1]);
    const double r2 = ((1.0 - su) * vu0[2] + su * vu1[2]) - ((1.0 - sw) * vw0[2] + sw * vw1[2]);
    const double vn = n0 * r0 + n1 * r1 + n2 * r2;
    const double fn = delta * (k - c * vn);
    if (!(fn > 0.0)) return dist;
    const double t0 = r0 - vn * n0, t1 = r1 - vn * n1, t2 = r2 - vn * n2;
    const double sp = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
    const double gf = mu * fn / (sp > vs ? sp : vs);
    double f0 = fn * n0 - gf * t0, f1 = fn * n1 - gf * t1, f2 = fn * n2 - gf * t2;   // on u
    double sp_ = su;
    if (!first) {
        f0 = -f0; f1 = -f1; f2 = -f2;
        sp_ = sw;
    }
    fa[0] += (1.0 - sp_) * f0; fa[1] += (1.0 - sp_) * f1; fa[2] += (1.0 - sp_) * f2;
    fb[0] += sp_ * f0; fb[1] += sp_ * f1; fb[2] += sp_ * f2;
    return dist;
}

// Verlet lists of capsules: element s's record for the pass, four double4 by
// slot: (A, radius), (B, rod), (v_A, element), (v_B, 0).
__device__ __attribute__((always_inline)) inline void element_record(const ContactGrid &G, int64_t s, double4 r[4])
{
    for (int k = 0; k < 4; ++k) r[k] = G.srec[4 * s + k];
}

// Element s's contacts over its list entries 0 .. n-1 (element slots), in
// list (increasing slot) order, two partners' records loaded at a time
// (entries past the end repeat the last one and are not evaluated).
__device__ __attribute__((always_inline)) inline void capsule_list(const ContactGrid &G, int64_t s, int n, const double4 me[4], double k, double c,
                                    double mu, double vs, double fa[3], double fb[3], double &pot)
{
    for (int j0 = 0; j0 < n; j0 += 2) {
        double4 q[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) element_record(G, G.lid[min(j0 + u, n - 1) * G.nn + s], q[u]);
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (j0 + u < n)
                capsule_pair(me[0], me[1], me[2], me[3], q[u][0], q[u][1], q[u][2], q[u][3], k, c, mu, vs, fa, fb,
                             pot);
    }
}

// Each element sums its contacts over the 27 buckets around its midpoint, in
// two phases so that the wave's lanes do the costly FP64 work together.  The
// screen: every candidate's capsule bounding box against the element's in
// FP32, four candidates' records loaded at a time and tested without
// branches, and elements of the same rod closer than the self-contact rule
// allows dropped; a survivor's sorted position goes to the lane's queue in
// LDS.  A lane screens until its queue is nearly full or its sweep ends; then
// the wave drains its queues, each lane taking its survivors in the order it
// queued them (the order of the sweep, so the sums are those of a single
// pass; each pair by capsule_pair), and lanes with candidates left go on.
template <typename T, bool LIST>
__global__ __launch_bounds__(CF_BLOCK) void seg_force_kernel(const DevBatch<T> B, const ContactGrid G, int nb,
                                                             Gate gate)
{
    if (gate.skip()) return;
    __shared__ int32_t queue[CF_QUEUE * CF_BLOCK];
    int32_t *const mine = queue + threadIdx.x;   // entry j at mine[j * CF_BLOCK]
    const int64_t p0 = blockIdx.x * (int64_t)CF_BLOCK + threadIdx.x;
    // no early exit: every lane reaches the wave-wide drains
    const bool live = p0 < G.start[nb];
    const int64_t pm = live ? p0 : 0;
    const double4 ua = G.sca[pm], ub = G.scb[pm], uva = G.sva[pm], uvb = G.svb[pm];
    const float4 mc = G.cull[2 * pm], me = G.cull[2 * pm + 1];
    const float mg = cull_margin(mc, (float)(1.0 / G.inv_cell));
    // own half extents plus the margin (building lists: plus the skin, so
    // boxes closer than the skin per axis pass)
    const float sk = LIST ? (float)G.skin : 0.0f;
    const float ex = mc.w + mg + sk, ey = me.x + mg + sk, ez = me.y + mg + sk;
    const int rod = (int)ub.w, elem = (int)uva.w;
    const int64_t sme = live ? G.sid[p0] : 0;
    // elements of the own rod it may touch: up to `prev` and from `next` on
    const int next = G.self_pairs[sme], prev = G.self_pairs[G.nn + sme];
    const double k = B.wall_k, c = B.wall_c, mu = B.wall_mu, vs = B.wall_vslip;
    double fa[3] = {0.0, 0.0, 0.0}, fb[3] = {0.0, 0.0, 0.0}, pot = 0;
    int nq = 0;

    auto evaluate = [&](int32_t p) {
        return capsule_pair(ua, ub, uva, uvb, G.sca[p], G.scb[p], G.sva[p], G.svb[p], k, c, mu, vs, fa, fb, pot);
    };
    // building lists: a pair joins when its segments are closer than the radii
    // plus the skin, plus a slack (0.1% of the skin and a millionth of a cell)
    // far above the computed distance's rounding, near-parallel segments'
    // included, whatever the skin
    const double reach = G.skin * (1.0 + 1e-3) + 1e-6 / G.inv_cell;
    int n_list = 0;
    const int64_t NN = G.nn;

    Sweep sw(G, cell_of(0.5 * (ua.x + ub.x), G.org[0], G.inv_cell), cell_of(0.5 * (ua.y + ub.y), G.org[1], G.inv_cell),
             cell_of(0.5 * (ua.z + ub.z), G.org[2], G.inv_cell));
    bool done = !live || !sw.next(G);
    for (;;) {
        while (!done && nq <= CF_QUEUE - CF_GROUP) {
            const float4 *const q = G.cull + 2 * (int64_t)sw.p;
            float4 q0[CF_GROUP], q1[CF_GROUP];
#pragma unroll
            for (int u = 0; u < CF_GROUP; ++u) {
                q0[u] = q[2 * u];
                q1[u] = q[2 * u + 1];
            }
#pragma unroll
            for (int u = 0; u < CF_GROUP; ++u) {
                // half extents: x in the first record's w, y and z in the second's x and y
                const bool box = (fabsf(mc.x - q0[u].x) < ex + q0[u].w) & (fabsf(mc.y - q0[u].y) < ey + q1[u].x)
                               & (fabsf(mc.z - q0[u].z) < ez + q1[u].y);
                const int qe = __float_as_int(q1[u].w);   // the element itself fails both bounds
                const bool pair = (__float_as_int(q1[u].z) != rod) | (qe >= next) | (qe <= prev);
                mine[nq * CF_BLOCK] = sw.p + u;   // nq < CF_QUEUE: a free slot, kept only if it passed
                nq += (int)((sw.p + u < sw.pe) & box & pair);
            }
            sw.p += CF_GROUP;
            if (sw.p >= sw.pe) done = !sw.next(G);
        }
        for (int j = 0; j < nq; ++j) {
            const int32_t p = mine[j * CF_BLOCK];
            const double dist = evaluate(p);
            if constexpr (LIST) {
                if (dist < ua.w + G.sca[p].w + reach) {
                    if (n_list < CONTACT_LIST_CAP) G.lid[n_list * NN + sme] = G.sid[p];
                    ++n_list;
                }
            }
        }
        nq = 0;
        if (!__any(!done)) break;
    }
    if constexpr (LIST) {
        int most = n_list;   // the wave's longest list, one atomic per wave
        for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o, 64));
        if ((threadIdx.x & 63) == 0 && most > 0) atomicMax(&G.vflag[VF_MOST], most);
        if (live) {
            G.lcount[sme] = n_list;
            if (n_list > CONTACT_LIST_CAP) {
                atomicOr(&G.vflag[VF_OVERFLOW], 1);   // forces of the sweep's order; the next pass builds again
            } else {
                int32_t *const L = G.lid + sme;   // insertion sort by slot
                for (int i = 1; i < n_list; ++i) {
                    const int32_t key = L[i * NN];
                    int j = i - 1;
                    while (j >= 0 && L[j * NN] > key) {
                        L[(j + 1) * NN] = L[j * NN];
                        --j;
                    }
                    L[(j + 1) * NN] = key;
                }
                double4 mr[4];
                element_record(G, sme, mr);
                for (int a = 0; a < 3; ++a) fa[a] = fb[a] = 0.0;
                pot = 0.0;
                capsule_list(G, sme, n_list, mr, k, c, mu, vs, fa, fb, pot);
            }
        }
    }
    if (!live) return;
    const int64_t s = G.sid[p0], nn = G.nn;
    for (int a = 0; a < 3; ++a) {
        G.fseg[a * nn + s] = fa[a];
        G.fseg[(3 + a) * nn + s] = fb[a];
    }
    G.pot[s] = pot;
}

// Verlet lists of capsules, first kernel of every pass: every element's
// record (above) and the move check of its node A, and of the rod's last node
// after its last element, so every node is checked once (as for node
// spheres: a node that moved more than half the skin asks for a build; the
// distance between two segments changes by at most the largest move of
// either's points, so no pair missing from the lists can touch).
template <typename T>
__global__ __launch_bounds__(256) void seg_pack_kernel(const DevBatch<T> B, const ContactGrid G, double drift)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, NI = G.nid;
    int moved = 0;
    if (s < G.nn) {
        int rod, elem;
        double a[3], b[3], va[3], vb[3];
        contact_segment(B, G, s, drift, rod, elem, a, b, va, vb);
        if (rod >= 0) {
            G.srec[4 * s] = make_double4(a[0], a[1], a[2], B.rod_rad[rod]);
            G.srec[4 * s + 1] = make_double4(b[0], b[1], b[2], (double)rod);
            G.srec[4 * s + 2] = make_double4(va[0], va[1], va[2], (double)elem);
            G.srec[4 * s + 3] = make_double4(vb[0], vb[1], vb[2], 0.0);
            const double h = 0.5 * G.skin;
            auto check = [&](const double x[3], int64_t id) {
                if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) return;   // a build records NaN there
                const double e0 = x[0] - G.xb[id], e1 = x[1] - G.xb[NI + id], e2 = x[2] - G.xb[2 * NI + id];
                moved |= !(e0 * e0 + e1 * e1 + e2 * e2 <= h * h);
            };
            check(a, s);
            if (elem + 1 == B.rod_n[rod]) check(b, B.n_slots + rod);
        }
    }
    if (__any(moved) && (threadIdx.x & 63) == 0) atomicOr(&G.vflag[VF_REQUEST], 1);
}

// Verlet lists of capsules, every pass: each element with partners sums its
// contacts over its list from the records; one without reads and writes
// nothing (its shares are the zeros the last build wrote).  With a build in
// this pass the shares computed here are replaced.
template <typename T>
__global__ __launch_bounds__(256) void seg_list_kernel(const DevBatch<T> B, const ContactGrid G)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, nn = G.nn;
    if (s >= nn) return;
    const int n = min(G.lcount[s], CONTACT_LIST_CAP);   // larger only after an overflow, when a build follows
    if (n == 0) return;
    double4 me[4];
    element_record(G, s, me);
    double fa[3] = {0.0, 0.0, 0.0}, fb[3] = {0.0, 0.0, 0.0}, pot = 0.0;
    capsule_list(G, s, n, me, B.wall_k, B.wall_c, B.wall_mu, B.wall_vslip, fa, fb, pot);
    for (int a = 0; a < 3; ++a) {
        G.fseg[a * nn + s] = fa[a];
        G.fseg[(3 + a) * nn + s] = fb[a];
    }
    G.pot[s] = pot;
}

// Node forces from the elements' shares: node i of a rod takes element i's
// A share and element i - 1's B share (node n: element n - 1's B share).
template <typename T>
__global__ void seg_nodes_kernel(const DevBatch<T> B, const ContactGrid G)
{
    const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (id >= G.nid) return;
    const int64_t NS = B.n_slots, nn = G.nn;
    int64_t sa = -1, sb = -1;   // elements whose A / B share lands here
    if (id < NS) {
        const int rod = B.slot_rod[id];
        if (rod < 0) return;
        sa = id;
        if (B.slot_idx[id] > 0) sb = id - 1;
    } else {
        const int rod = (int)(id - NS);
        sb = B.rod_slot[rod] + B.rod_n[rod] - 1;
    }
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        if (sa >= 0) f[a] += G.fseg[a * nn + sa];
        if (sb >= 0) f[a] += G.fseg[(3 + a) * nn + sb];
        G.force[a * G.nid + id] = f[a];
    }
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
        if ((!g.xabs && !g.rec) || !g.origin) return hipErrorInvalidValue;
        hipLaunchKernelGGL(contact_positions_kernel, dim3((b.n_rods + 3) / 4), dim3(256), 0, s, b, g, drift);
    }
    const bool seg = g.mode == 2;
    if (seg ? (!g.sca || !g.fseg || !g.self_pairs || !g.cull) : !g.spr) return hipErrorInvalidValue;
    const bool lists = g.skin > 0.0;
    if (lists && (!g.lcount || !g.lid || !g.xb || !g.vflag || (seg ? !g.srec : !g.rec))) return hipErrorInvalidValue;
    const unsigned gf = (unsigned)((g.nn + CF_BLOCK - 1) / CF_BLOCK);
    Gate build;   // with lists the grid pass runs only in passes that rebuild them
    if (lists) {
        build.p = g.vflag + VF_REQUEST;
        if (seg) {
            hipLaunchKernelGGL((seg_pack_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift);
            hipLaunchKernelGGL((seg_list_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g);
        } else {
            const dim3 gi((unsigned)((g.nid + bs - 1) / bs));
            // FP32 batches: the positions kernel above wrote the records
            if constexpr (sizeof(T) == 8) hipLaunchKernelGGL((verlet_pack_kernel<T>), gi, dim3(bs), 0, s, b, g, drift);
            hipLaunchKernelGGL((verlet_force_kernel<T>), gi, dim3(bs), 0, s, b, g);
        }
    }
    if (seg) hipLaunchKernelGGL((seg_bin_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift, build);
    else hipLaunchKernelGGL((contact_bin_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift, build);
    hipLaunchKernelGGL(contact_scan_chunks, dim3(n_chunks), dim3(256), 0, s, g, nb, build);
    hipLaunchKernelGGL(contact_scan_top, dim3(1), dim3(1024), 0, s, g, n_chunks, nb, build);
    hipLaunchKernelGGL(contact_scan_add, dim3(n_chunks), dim3(256), 0, s, g, nb, build);
    if (seg) {
        hipLaunchKernelGGL(contact_scatter_ids, dim3(gn), dim3(bs), 0, s, g, build);
        hipLaunchKernelGGL(sort_ids_kernel, dim3(gn), dim3(bs), 0, s, g, build);
        hipLaunchKernelGGL((seg_fill_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift, nb, build);
        if (lists)
            hipLaunchKernelGGL((seg_force_kernel<T, true>), dim3(gf), dim3(CF_BLOCK), 0, s, b, g, nb, build);
        else
            hipLaunchKernelGGL((seg_force_kernel<T, false>), dim3(gf), dim3(CF_BLOCK), 0, s, b, g, nb, build);
        hipLaunchKernelGGL((seg_nodes_kernel<T>), dim3((unsigned)((g.nid + bs - 1) / bs)), dim3(bs), 0, s, b, g);
    } else {
        hipLaunchKernelGGL((contact_scatter_kernel<T>), dim3(gn), dim3(bs), 0, s, b, g, drift, build);
        hipLaunchKernelGGL(contact_sort_kernel, dim3(gn), dim3(bs), 0, s, g, build);
        if (lists)
            hipLaunchKernelGGL((contact_force_kernel<T, true>), dim3(gf), dim3(CF_BLOCK), 0, s, b, g, nb, drift,
                               build);
        else
            hipLaunchKernelGGL((contact_force_kernel<T, false>), dim3(gf), dim3(CF_BLOCK), 0, s, b, g, nb, drift,
                               build);
    }
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

hipError_t launch_contact_finish(const ContactGrid &g, int64_t *step, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(verlet_finish_kernel, dim3(1), dim3(64), 0, s, g.vflag, step, n);
    return hipGetLastError();
}

}  // namespace rodk
