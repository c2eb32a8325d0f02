// rod_lib.cpp -- host runtime behind include/rod.h: argument checks, the
// derived per-element constants (FP64), packing of whole rods into
// workgroup tiles, HIP-graph capture of the launch sequence, state I/O.
//
// Constitutive and inertial constants follow Elastica++, Methods, "Cosserat
// rod dynamics": S = diag(alpha_c G A, alpha_c G A, E A),
// B = diag(E I1, E I2, G (I1 + I2)), inertia rho I per unit length, for a
// solid circular section A = pi r^2, I1 = I2 = pi r^4 / 4.
#include "rod.h"
#include "rod_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? ROD_ENOMEM : ROD_EDEVICE,                \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

struct HostInputs {
    std::vector<int32_t> n;
    std::vector<double> pos, vel, dir, om, lh, k0;
    std::vector<double> rho, E, G, rad, ac, gam;
    std::vector<int32_t> bc0, bc1;
    std::vector<double> fend, camp, cfreq, cphase;
    std::vector<double> mag;     // [N_e][3] magnetization per unit length (empty: none)
    std::vector<double> mamp, maxis, mfreq, mwave, mphase;   // muscle torques (empty: none)
    std::vector<int32_t> crod, cnode;                        // connections [C][2] (empty: none)
    std::vector<double> ck, cc, crest;
    bool has_k0 = false, has_f = false, has_c = false;
};

template <typename X>
int fetch(std::vector<X> &dst, const X *src, size_t count, bool on_device)
{
    dst.resize(count);
    if (count == 0) return ROD_OK;
    if (on_device) {
        HIPCHK(hipMemcpy(dst.data(), src, count * sizeof(X), hipMemcpyDeviceToHost));
    } else {
        std::memcpy(dst.data(), src, count * sizeof(X));
    }
    return ROD_OK;
}

}  // namespace

int rodk::set_error(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

struct rod_batch {
    int precision = ROD_F64;
    int waves = 1;
    int substeps = 0;
    int grid = 0;
    int32_t R = 0;
    int64_t Ne = 0, Nn = 0, n_slots = 0;
    int n_tiles = 0;
    double dt = 0, t0 = 0;
    int64_t steps = 0;           // steps since t0 (mirrors the device counter)
    std::vector<int32_t> n;
    std::vector<int32_t> rod_slot;
    std::vector<double> origin;  // [R][3]
    // clamped ends: creation values of node 0 / element 0 and node n / element n-1
    std::vector<int32_t> bc0, bc1;
    std::vector<double> clamp_r0, clamp_q0, clamp_rn, clamp_qn;   // [R][3], [R][9]
    std::vector<double> E, G, rho, rad, ac, camp, cfreq, cphase;  // per-rod inputs kept for the surrogate
    bool magnetic = false, muscle = false;
    bool ext = false;            // magnetic, gravity or muscle: the step runs the extended kernel
    double field[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, field_freq = 0;
    double grav[3] = {0, 0, 0};
    // device
    void *d_state = nullptr, *d_param = nullptr, *d_tail = nullptr, *d_rodp = nullptr;
    void *d_mag = nullptr;       // [3][n_slots] magnetization times rest length (magnetic batches)
    void *d_mus = nullptr;       // [3][n_slots] muscle amplitude times axis at the slot's Voronoi point
    double *d_mus_ofs = nullptr; // [n_slots] muscle phase offset phi - q s_k
    double *d_mus_freq = nullptr;   // [R] muscle frequency
    double *d_grav_r0 = nullptr;    // [3][n_slots + R] creation positions (batches with gravity)
    // connections: per-slot compact node indices, CSR over them, spring parameters, rod offsets
    int32_t *d_conn_idx = nullptr;  // [2][n_slots]
    int32_t *d_conn_off = nullptr;  // [total + 1]
    int32_t *d_conn_tbase = nullptr;   // [n_tiles] first compact index of each tile
    int32_t *d_conn_partner = nullptr; // [2C] partner's compact index within its tile
    int32_t *d_conn_key = nullptr;     // [total] slot * 2 + column of each compact index
    double *d_conn_par = nullptr;      // [3][2C] k, c, rest
    double *d_rod_org = nullptr;       // [3][R] rod origins (connections or walls)
    double *d_rod_rad = nullptr;       // [R] rod radii (walls)
    void *d_wall_off = nullptr;        // [n_tiles][8] wall offsets in each tile's frame
    int n_walls = 0;
    bool rod_contact = false;          // rod-rod contact: a grid pass before every step
    int contact_mode = 0;              // 1: node spheres, 2: element capsules
    double contact_skin = 0;           // as given (mode 1: < 0 no Verlet lists, 0 a fifth of the largest radius)
    rodk::ContactGrid cg{};
    double walls[ROD_MAX_WALLS][4] = {};
    double wall_k = 0, wall_c = 0, wall_mu = 0, wall_vslip = 0;
    int conn_max_nodes = 0;            // most connected nodes in one tile
    int n_conn = 0;
    double *d_freq = nullptr, *d_phase = nullptr, *d_energy = nullptr;
    int32_t *d_ints = nullptr;   // slot_rod, slot_idx, rod_n, rod_flags, rod_slot, nonfinite
    int64_t *d_step = nullptr;
    rodk::DevBatch<double> b64{};
    rodk::DevBatch<float> b32{};
    hipStream_t capture_stream = nullptr;
    std::map<int64_t, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    bool use_graphs = true;
    std::vector<rod_tune_trial> tune_log;   // autotuner trials (empty without autotuning)
    // host staging of the packed layout
    std::vector<int32_t> slot_rod, slot_idx;
};

namespace {

static_assert(ROD_MAX_WALLS == rodk::DEV_MAX_WALLS, "the device batch holds ROD_MAX_WALLS walls");

size_t elem_bytes(const rod_batch *b) { return b->precision == ROD_F32 ? 4 : 8; }

// Groups of rods joined (directly or through other rods) by connections; a
// rod without connections is a group of its own.  Members in rod order.
std::vector<std::vector<int32_t>> connected_groups(int R, const std::vector<int32_t> &crod)
{
    std::vector<int32_t> parent(R);
    for (int r = 0; r < R; ++r) parent[r] = r;
    auto root = [&](int32_t x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
    };
    for (size_t c = 0; c + 1 < crod.size(); c += 2) {
        const int32_t a = root(crod[c]), b = root(crod[c + 1]);
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
    std::vector<int32_t> gid(R, -1);
    std::vector<std::vector<int32_t>> groups;
    for (int r = 0; r < R; ++r) {
        const int32_t g = root(r);
        if (gid[g] < 0) {
            gid[g] = (int32_t)groups.size();
            groups.emplace_back();
        }
        groups[gid[g]].push_back(r);
    }
    return groups;
}

// Best-fit decreasing packing of whole groups into tiles of `cap` lanes; the
// rods of a group sit on consecutive lanes of one tile.
void pack_tiles(const std::vector<int32_t> &n, const std::vector<std::vector<int32_t>> &groups, int cap,
                std::vector<int32_t> &rod_slot, int &n_tiles)
{
    const int G = (int)groups.size();
    std::vector<int> size(G, 0);
    for (int g = 0; g < G; ++g)
        for (int32_t r : groups[g]) size[g] += n[r];
    std::vector<int32_t> order(G);
    for (int g = 0; g < G; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size[a] > size[b]; });
    std::multiset<std::pair<int, int>> room;   // (free lanes, tile)
    std::vector<int> used;
    rod_slot.assign(n.size(), 0);
    for (int g : order) {
        auto it = room.lower_bound({size[g], -1});
        int tile;
        if (it == room.end()) {
            tile = (int)used.size();
            used.push_back(0);
        } else {
            tile = it->second;
            room.erase(it);
        }
        for (int32_t r : groups[g]) {
            rod_slot[r] = tile * cap + used[tile];
            used[tile] += n[r];
        }
        if (cap - used[tile] > 0) room.insert({cap - used[tile], tile});
    }
    n_tiles = (int)used.size();
}

int validate(const rod_batch_desc *d)
{
    if (!d) return fail(ROD_EINVAL, "desc is NULL");
    if (d->n_rods < 1) return fail(ROD_EINVAL, "n_rods must be >= 1");
    if (!d->n_elems || !d->position || !d->velocity || !d->director || !d->omega || !d->density
        || !d->youngs || !d->shear_modulus || !d->radius || !d->shear_coeff)
        return fail(ROD_EINVAL, "a required array is NULL");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(ROD_EINVAL, "dt must be > 0");
    if (!std::isfinite(d->t0)) return fail(ROD_EINVAL, "t0 must be finite");
    if (d->precision != ROD_F64 && d->precision != ROD_F32) return fail(ROD_EINVAL, "precision must be ROD_F64 or ROD_F32");
    if (d->substeps < 0) return fail(ROD_EINVAL, "substeps must be >= 0");
    if (d->tile_waves != 0 && d->tile_waves != 1 && d->tile_waves != 2 && d->tile_waves != 4 && d->tile_waves != 8)
        return fail(ROD_EINVAL, "tile_waves must be 0, 1, 2, 4 or 8");
    if (d->autotune != 0 && d->autotune != 1) return fail(ROD_EINVAL, "autotune must be 0 or 1");
    if (d->couple_amp && (!d->couple_freq || !d->couple_phase))
        return fail(ROD_EINVAL, "couple_amp needs couple_freq and couple_phase");
    if (d->magnetization) {
        for (int k = 0; k < 9; ++k)
            if (!std::isfinite(d->field[k])) return fail(ROD_EINVAL, "field is not finite");
        if (!std::isfinite(d->field_freq)) return fail(ROD_EINVAL, "field_freq is not finite");
    }
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(d->gravity[k])) return fail(ROD_EINVAL, "gravity is not finite");
    if (d->muscle_amp && (!d->muscle_axis || !d->muscle_freq || !d->muscle_wavenumber || !d->muscle_phase))
        return fail(ROD_EINVAL, "muscle_amp needs muscle_axis, muscle_freq, muscle_wavenumber and muscle_phase");
    if (d->n_connections < 0) return fail(ROD_EINVAL, "n_connections must be >= 0");
    if (d->n_connections > 0 && (!d->conn_rod || !d->conn_node || !d->conn_k || !d->conn_c || !d->conn_rest))
        return fail(ROD_EINVAL, "connections need conn_rod, conn_node, conn_k, conn_c and conn_rest");
    if (d->n_walls < 0 || d->n_walls > ROD_MAX_WALLS)
        return fail(ROD_EINVAL, "n_walls must be in [0, " + std::to_string(ROD_MAX_WALLS) + "]");
    if (d->rod_contact < 0 || d->rod_contact > 2) return fail(ROD_EINVAL, "rod_contact must be 0, 1 or 2");
    if (d->rod_contact && d->substeps > 1)
        return fail(ROD_EINVAL, "rod contact runs one step per launch: substeps must be 0 or 1");
    if (!std::isfinite(d->contact_skin)) return fail(ROD_EINVAL, "contact_skin must be finite");
    if (d->n_walls > 0 || d->rod_contact) {
        if (d->n_walls > 0 && !d->walls) return fail(ROD_EINVAL, "walls is NULL");
        for (int w = 0; w < d->n_walls; ++w) {
            const double *n = &d->walls[4 * w];
            for (int k = 0; k < 4; ++k)
                if (!std::isfinite(n[k])) return fail(ROD_EINVAL, "wall " + std::to_string(w) + " is not finite");
            if (std::fabs(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] - 1.0) > 1e-9)
                return fail(ROD_EINVAL, "wall " + std::to_string(w) + ": the normal must be a unit vector");
        }
        if (!(d->wall_k >= 0) || !(d->wall_c >= 0) || !(d->wall_mu >= 0) || !std::isfinite(d->wall_k)
            || !std::isfinite(d->wall_c) || !std::isfinite(d->wall_mu))
            return fail(ROD_EINVAL, "wall_k, wall_c and wall_mu must be finite and >= 0");
        if (!(d->wall_vslip > 0) || !std::isfinite(d->wall_vslip)) return fail(ROD_EINVAL, "wall_vslip must be > 0");
    }
    return ROD_OK;
}

int gather_inputs(const rod_batch_desc *d, HostInputs &h)
{
    const bool dev = d->inputs_on_device != 0;
    const int R = d->n_rods;
    int rc;
    if ((rc = fetch(h.n, d->n_elems, R, dev))) return rc;
    int64_t Ne = 0;
    for (int r = 0; r < R; ++r) {
        if (h.n[r] < 1 || h.n[r] > ROD_MAX_ELEMS)
            return fail(ROD_EINVAL, "rod " + std::to_string(r) + ": n_elems " + std::to_string(h.n[r])
                                        + " outside [1, " + std::to_string(ROD_MAX_ELEMS) + "]");
        Ne += h.n[r];
    }
    const int64_t Nn = Ne + R, Nv = Ne - R;
    if ((rc = fetch(h.pos, d->position, 3 * Nn, dev))) return rc;
    if ((rc = fetch(h.vel, d->velocity, 3 * Nn, dev))) return rc;
    if ((rc = fetch(h.dir, d->director, 9 * Ne, dev))) return rc;
    if ((rc = fetch(h.om, d->omega, 3 * Ne, dev))) return rc;
    if (d->rest_length) {
        if ((rc = fetch(h.lh, d->rest_length, Ne, dev))) return rc;
    }
    if (d->rest_kappa) {
        if ((rc = fetch(h.k0, d->rest_kappa, 3 * Nv, dev))) return rc;
        h.has_k0 = true;
    }
    if ((rc = fetch(h.rho, d->density, R, dev))) return rc;
    if ((rc = fetch(h.E, d->youngs, R, dev))) return rc;
    if ((rc = fetch(h.G, d->shear_modulus, R, dev))) return rc;
    if ((rc = fetch(h.rad, d->radius, R, dev))) return rc;
    if ((rc = fetch(h.ac, d->shear_coeff, R, dev))) return rc;
    if (d->damping) {
        if ((rc = fetch(h.gam, d->damping, R, dev))) return rc;
    } else {
        h.gam.assign(R, 0.0);
    }
    if (d->bc_start) {
        if ((rc = fetch(h.bc0, d->bc_start, R, dev))) return rc;
    } else {
        h.bc0.assign(R, 0);
    }
    if (d->bc_end) {
        if ((rc = fetch(h.bc1, d->bc_end, R, dev))) return rc;
    } else {
        h.bc1.assign(R, 0);
    }
    if (d->end_force) {
        if ((rc = fetch(h.fend, d->end_force, 3 * R, dev))) return rc;
        h.has_f = true;
    } else {
        h.fend.assign(3 * R, 0.0);
    }
    if (d->couple_amp) {
        if ((rc = fetch(h.camp, d->couple_amp, 3 * R, dev))) return rc;
        if ((rc = fetch(h.cfreq, d->couple_freq, R, dev))) return rc;
        if ((rc = fetch(h.cphase, d->couple_phase, R, dev))) return rc;
        h.has_c = true;
    } else {
        h.camp.assign(3 * R, 0.0);
        h.cfreq.assign(R, 0.0);
        h.cphase.assign(R, 0.0);
    }
    if (d->magnetization) {
        if ((rc = fetch(h.mag, d->magnetization, 3 * Ne, dev))) return rc;
    }
    if (d->n_connections > 0) {
        const size_t C = (size_t)d->n_connections;
        if ((rc = fetch(h.crod, d->conn_rod, 2 * C, dev))) return rc;
        if ((rc = fetch(h.cnode, d->conn_node, 2 * C, dev))) return rc;
        if ((rc = fetch(h.ck, d->conn_k, C, dev))) return rc;
        if ((rc = fetch(h.cc, d->conn_c, C, dev))) return rc;
        if ((rc = fetch(h.crest, d->conn_rest, C, dev))) return rc;
    }
    if (d->muscle_amp) {
        if ((rc = fetch(h.mamp, d->muscle_amp, Nv, dev))) return rc;
        if ((rc = fetch(h.maxis, d->muscle_axis, 3 * R, dev))) return rc;
        if ((rc = fetch(h.mfreq, d->muscle_freq, R, dev))) return rc;
        if ((rc = fetch(h.mwave, d->muscle_wavenumber, R, dev))) return rc;
        if ((rc = fetch(h.mphase, d->muscle_phase, R, dev))) return rc;
    }
    return ROD_OK;
}

int check_values(HostInputs &h)
{
    const int R = (int)h.n.size();
    for (int r = 0; r < R; ++r) {
        const std::string tag = "rod " + std::to_string(r) + ": ";
        if (!(h.rho[r] > 0) || !(h.E[r] > 0) || !(h.G[r] > 0) || !(h.rad[r] > 0) || !(h.ac[r] > 0))
            return fail(ROD_EINVAL, tag + "density, youngs, shear_modulus, radius and shear_coeff must be > 0");
        if (!(h.gam[r] >= 0) || !std::isfinite(h.gam[r])) return fail(ROD_EINVAL, tag + "damping must be >= 0");
        if ((h.bc0[r] != 0 && h.bc0[r] != 1) || (h.bc1[r] != 0 && h.bc1[r] != 1))
            return fail(ROD_EINVAL, tag + "bc flags must be ROD_FREE or ROD_CLAMPED");
    }
    for (double x : h.pos) if (!std::isfinite(x)) return fail(ROD_EINVAL, "position is not finite");
    for (double x : h.vel) if (!std::isfinite(x)) return fail(ROD_EINVAL, "velocity is not finite");
    for (double x : h.om) if (!std::isfinite(x)) return fail(ROD_EINVAL, "omega is not finite");
    for (double x : h.mag) if (!std::isfinite(x)) return fail(ROD_EINVAL, "magnetization is not finite");
    for (const auto *vec : {&h.mamp, &h.maxis, &h.mfreq, &h.mwave, &h.mphase})
        for (double x : *vec) if (!std::isfinite(x)) return fail(ROD_EINVAL, "a muscle input is not finite");
    for (size_t c = 0; c < h.ck.size(); ++c) {
        const std::string tag = "connection " + std::to_string(c) + ": ";
        for (int end = 0; end < 2; ++end) {
            const int32_t r = h.crod[2 * c + end], j = h.cnode[2 * c + end];
            if (r < 0 || r >= R) return fail(ROD_EINVAL, tag + "rod outside the batch");
            if (j < 0 || j > h.n[r]) return fail(ROD_EINVAL, tag + "node outside its rod");
        }
        if (h.crod[2 * c] == h.crod[2 * c + 1] && h.cnode[2 * c] == h.cnode[2 * c + 1])
            return fail(ROD_EINVAL, tag + "joins a node to itself");
        if (!(h.ck[c] >= 0) || !(h.cc[c] >= 0) || !(h.crest[c] >= 0) || !std::isfinite(h.ck[c])
            || !std::isfinite(h.cc[c]) || !std::isfinite(h.crest[c]))
            return fail(ROD_EINVAL, tag + "k, c and l0 must be finite and >= 0");
    }
    const int64_t Ne = (int64_t)h.dir.size() / 9;
    for (int64_t i = 0; i < Ne; ++i) {
        const double *q = &h.dir[9 * i];
        double worst = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = q[3 * a] * q[3 * b] + q[3 * a + 1] * q[3 * b + 1] + q[3 * a + 2] * q[3 * b + 2];
                worst = std::max(worst, std::fabs(s - (a == b ? 1.0 : 0.0)));
            }
        const double det = q[0] * (q[4] * q[8] - q[5] * q[7]) - q[1] * (q[3] * q[8] - q[5] * q[6])
                         + q[2] * (q[3] * q[7] - q[4] * q[6]);
        if (!(worst <= 1e-8) || !(det > 0))
            return fail(ROD_EINVAL, "director of element " + std::to_string(i) + " is not in SO(3) within 1e-8");
    }
    // rest lengths: given or the initial chord lengths
    const bool given = !h.lh.empty();
    if (!given) h.lh.resize(Ne);
    int64_t e = 0, nd = 0;
    for (int r = 0; r < R; ++r) {
        for (int i = 0; i < h.n[r]; ++i, ++e) {
            const double *a = &h.pos[3 * (nd + i)], *b = &h.pos[3 * (nd + i + 1)];
            const double l = std::sqrt((b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1])
                                       + (b[2] - a[2]) * (b[2] - a[2]));
            if (!(l > 0)) return fail(ROD_EINVAL, "element " + std::to_string(e) + " has zero length");
            if (!given) h.lh[e] = l;
            if (!(h.lh[e] > 0) || !std::isfinite(h.lh[e]))
                return fail(ROD_EINVAL, "rest length of element " + std::to_string(e) + " must be > 0");
        }
        nd += h.n[r] + 1;
    }
    return ROD_OK;
}

// Crude explicit stability bound: 2 / (largest natural frequency) over the
// axial, shear, bending, twisting and rotational-shear modes of one element.
double stability_dt(const HostInputs &h, const double *field, double wall_k = 0.0, double contact_k = 0.0)
{
    double dt = 1e300;
    double bmax = 0;   // bound on |b(t)|
    if (!h.mag.empty())
        for (int c = 0; c < 3; ++c)
            bmax += std::sqrt(field[3 * c] * field[3 * c] + field[3 * c + 1] * field[3 * c + 1]
                              + field[3 * c + 2] * field[3 * c + 2]);
    int64_t e = 0;
    for (size_t r = 0; r < h.n.size(); ++r) {
        double lmin = 1e300, mmax = 0;
        for (int i = 0; i < h.n[r]; ++i) {
            lmin = std::min(lmin, h.lh[e + i]);
            if (!h.mag.empty())
                mmax = std::max(mmax, std::sqrt(h.mag[3 * (e + i)] * h.mag[3 * (e + i)]
                                                + h.mag[3 * (e + i) + 1] * h.mag[3 * (e + i) + 1]
                                                + h.mag[3 * (e + i) + 2] * h.mag[3 * (e + i) + 2]));
        }
        e += h.n[r];
        const double A = M_PI * h.rad[r] * h.rad[r], I = M_PI * std::pow(h.rad[r], 4) / 4.0;
        const double rho = h.rho[r];
        double w = 0;
        w = std::max(w, 2.0 / lmin * std::sqrt(h.E[r] / rho));                       // axial
        w = std::max(w, 2.0 / lmin * std::sqrt(h.ac[r] * h.G[r] / rho));             // shear
        w = std::max(w, 4.0 / (lmin * lmin) * std::sqrt(h.E[r] * I / (rho * A)));    // bending
        w = std::max(w, 2.0 / lmin * std::sqrt(h.G[r] / rho));                       // twist
        w = std::max(w, std::sqrt(2.0 * h.ac[r] * h.G[r] * A / (rho * I)));          // rotational shear
        w = std::max(w, std::sqrt(mmax * bmax / (rho * I)));                         // magnetic restoring couple
        w = std::max(w, std::sqrt(wall_k / (0.5 * rho * A * lmin)));                // wall contact of an end node
        w = std::max(w, std::sqrt(2.0 * contact_k / (0.5 * rho * A * lmin)));       // two end nodes in contact
        dt = std::min(dt, 2.0 / w);
    }
    return dt;
}

template <typename T>
void fill_dev(rodk::DevBatch<T> &d, rod_batch *b)
{
    const int64_t NS = b->n_slots;
    d.state = (T *)b->d_state;
    d.param = (T *)b->d_param;
    d.tail = (T *)b->d_tail;
    d.rodp = (T *)b->d_rodp;
    d.rod_freq = b->d_freq;
    d.rod_phase = b->d_phase;
    d.slot_rod = b->d_ints;
    d.slot_idx = b->d_ints + NS;
    d.rod_n = b->d_ints + 2 * NS;
    d.rod_flags = d.rod_n + b->R;
    d.rod_slot = d.rod_flags + b->R;
    d.nonfinite = d.rod_slot + b->R;
    d.step = b->d_step;
    d.n_slots = NS;
    d.n_rods = b->R;
    d.n_tiles = b->n_tiles;
    d.dt = b->dt;
    d.t0 = b->t0;
    d.mag = (T *)b->d_mag;
    for (int k = 0; k < 9; ++k) d.field[k] = T(b->field[k]);
    d.field_freq = b->field_freq;
    d.field_ds = std::sin(2.0 * M_PI * b->field_freq * b->dt);
    d.field_dc = std::cos(2.0 * M_PI * b->field_freq * b->dt);
    d.ext = b->ext;
    for (int a = 0; a < 3; ++a) d.grav[a] = T(b->grav[a]);
    d.mus = (T *)b->d_mus;
    d.mus_ofs = b->d_mus_ofs;
    d.mus_freq = b->d_mus_freq;
    d.grav_r0 = b->d_grav_r0;
    d.conn_idx = b->d_conn_idx;
    d.conn_tbase = b->d_conn_tbase;
    d.conn_off = b->d_conn_off;
    d.conn_partner = b->d_conn_partner;
    d.conn_key = b->d_conn_key;
    d.conn_par = b->d_conn_par;
    d.rod_org = b->d_rod_org;
    d.rod_rad = b->d_rod_rad;
    d.wall_off = (const T *)b->d_wall_off;
    d.cforce = b->rod_contact ? b->cg.force : nullptr;
    d.cpot = b->rod_contact ? b->cg.pot : nullptr;
    d.n_walls = b->n_walls;
    for (int w = 0; w < 8; ++w)
        for (int k = 0; k < 4; ++k) d.wall[w][k] = T(w < b->n_walls ? b->walls[w][k] : 0.0);
    d.wall_k = T(b->wall_k);
    d.wall_c = T(b->wall_c);
    d.wall_mu = T(b->wall_mu);
    d.wall_vslip = T(b->wall_vslip);
    d.conn_nodes = b->conn_max_nodes;
    d.conn_entries = 2 * (int64_t)b->n_conn;
}

// Pack the dynamic state into the slot layout, imposing the clamped ends'
// constraints.  FP64 stores node positions; FP32 stores element edge vectors
// r_{i+1} - r_i (differences taken in FP64) and node 0 relative to the rod
// origin in the tail position fields.
template <typename T>
void pack_state(const rod_batch *b, const double *pos, const double *vel, const double *dir,
                const double *om, std::vector<T> &state, std::vector<T> &tail)
{
    constexpr bool EDGE = sizeof(T) == 4;
    const int64_t NS = b->n_slots;
    const int R = b->R;
    state.assign((size_t)rodk::N_STATE * NS, T(0));
    tail.assign((size_t)rodk::N_TAIL * R, T(0));
    // padding lanes: identity frames and unit-length elements (positions one
    // apart along z, or unit edges), so they stay finite and never feed
    // NaN/Inf to a neighbouring rod through the lane exchanges
    const int TL = 64 * b->waves;
    for (int64_t s = 0; s < NS; ++s) {
        state[rodk::Q00 * NS + s] = T(1);
        state[rodk::Q11 * NS + s] = T(1);
        state[rodk::Q22 * NS + s] = T(1);
        state[rodk::RZ * NS + s] = EDGE ? T(1) : T(1 + s % TL);
    }
    std::vector<double> x;
    int64_t e = 0, nd = 0;
    for (int r = 0; r < R; ++r) {
        const int n = b->n[r];
        const double *o = &b->origin[3 * r];
        // node positions with the clamped nodes at their creation values
        x.assign(&pos[3 * nd], &pos[3 * (nd + n + 1)]);
        if (b->bc0[r]) for (int a = 0; a < 3; ++a) x[a] = b->clamp_r0[3 * r + a];
        if (b->bc1[r]) for (int a = 0; a < 3; ++a) x[3 * n + a] = b->clamp_rn[3 * r + a];
        for (int i = 0; i < n; ++i) {
            const int64_t s = b->rod_slot[r] + i;
            const bool fixed_node = (i == 0 && b->bc0[r]);
            const bool fixed_elem = (i == 0 && b->bc0[r]) || (i == n - 1 && b->bc1[r]);
            for (int a = 0; a < 3; ++a) {
                state[(rodk::RX + a) * NS + s] = EDGE ? T(x[3 * (i + 1) + a] - x[3 * i + a]) : T(x[3 * i + a] - o[a]);
                state[(rodk::VX + a) * NS + s] = fixed_node ? T(0) : T(vel[3 * (nd + i) + a]);
                state[(rodk::WX + a) * NS + s] = fixed_elem ? T(0) : T(om[3 * (e + i) + a]);
            }
            const double *q = (i == 0 && b->bc0[r]) ? &b->clamp_q0[9 * r]
                            : (i == n - 1 && b->bc1[r]) ? &b->clamp_qn[9 * r] : &dir[9 * (e + i)];
            for (int k = 0; k < 9; ++k) state[(rodk::Q00 + k) * NS + s] = T(q[k]);
        }
        for (int a = 0; a < 3; ++a) {
            tail[(rodk::TRX + a) * R + r] = EDGE ? T(x[a] - o[a]) : T(x[3 * n + a] - o[a]);
            tail[(rodk::TVX + a) * R + r] = b->bc1[r] ? T(0) : T(vel[3 * (nd + n) + a]);
        }
        e += n;
        nd += n + 1;
    }
}

template <typename T>
int upload_state(rod_batch *b, const double *pos, const double *vel, const double *dir, const double *om)
{
    std::vector<T> state, tail;
    pack_state<T>(b, pos, vel, dir, om, state, tail);
    HIPCHK(hipMemcpy(b->d_state, state.data(), state.size() * sizeof(T), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_tail, tail.data(), tail.size() * sizeof(T), hipMemcpyHostToDevice));
    return ROD_OK;
}

template <typename T>
int build_device(rod_batch *b, const HostInputs &h)
{
    const int64_t NS = b->n_slots;
    const int R = b->R;
    // ---- per-slot constants (FP64 derivation, stored in T)
    std::vector<T> param((size_t)rodk::N_PARAM * NS, T(0));
    for (int64_t s = 0; s < NS; ++s) {   // padding: harmless values
        param[rodk::P_INV_M * NS + s] = T(0);
        param[rodk::P_LH * NS + s] = T(1);
        param[rodk::P_INV_LH * NS + s] = T(1);
        param[rodk::P_J1 * NS + s] = T(1);
        param[rodk::P_DH * NS + s] = T(1);
        param[rodk::P_INV_DH * NS + s] = T(1);
    }
    std::vector<T> rodp((size_t)rodk::N_RODP * R, T(0));
    std::vector<double> freq(R), phase(R);
    std::vector<int32_t> flags(R);
    int64_t e = 0, v = 0, nd = 0;
    for (int r = 0; r < R; ++r) {
        const int n = h.n[r];
        const double A = M_PI * h.rad[r] * h.rad[r];
        const double I = M_PI * std::pow(h.rad[r], 4) / 4.0;
        const double S1 = h.ac[r] * h.G[r] * A, S3 = h.E[r] * A;
        const double B1 = h.E[r] * I, B3 = h.G[r] * 2.0 * I;
        const double *lh = &h.lh[e];
        for (int i = 0; i < n; ++i) {
            const int64_t s = b->rod_slot[r] + i;
            const double m = 0.5 * h.rho[r] * A * ((i > 0 ? lh[i - 1] : 0.0) + lh[i]);
            param[rodk::P_INV_M * NS + s] = T(1.0 / m);
            param[rodk::P_LH * NS + s] = T(lh[i]);
            param[rodk::P_INV_LH * NS + s] = T(1.0 / lh[i]);
            param[rodk::P_J1 * NS + s] = T(h.rho[r] * I * lh[i]);
            param[rodk::P_S1 * NS + s] = T(S1);
            param[rodk::P_S3 * NS + s] = T(S3);
            if (i == 0) {
                // no Voronoi point left of the first element: finite placeholders
                // (its stiffness is zero)
                param[rodk::P_DH * NS + s] = T(lh[0]);
                param[rodk::P_INV_DH * NS + s] = T(1.0 / lh[0]);
            } else {
                // Voronoi point i-1, between elements i-1 and i, lives on slot i;
                // rest-length weighted stiffness of the two elements (equal material here)
                const double Dh = 0.5 * (lh[i - 1] + lh[i]);
                param[rodk::P_DH * NS + s] = T(Dh);
                param[rodk::P_INV_DH * NS + s] = T(1.0 / Dh);
                param[rodk::P_B1 * NS + s] = T((B1 * lh[i - 1] + B1 * lh[i]) / (lh[i - 1] + lh[i]));
                param[rodk::P_B3 * NS + s] = T((B3 * lh[i - 1] + B3 * lh[i]) / (lh[i - 1] + lh[i]));
                if (h.has_k0)
                    for (int a = 0; a < 3; ++a) param[(rodk::P_K0X + a) * NS + s] = T(h.k0[3 * (v + i - 1) + a]);
            }
        }
        const double mt = 0.5 * h.rho[r] * A * lh[n - 1];
        rodp[rodk::R_GAMMA * R + r] = T(h.gam[r]);
        rodp[rodk::R_INV_M_TAIL * R + r] = T(1.0 / mt);
        for (int a = 0; a < 3; ++a) {
            rodp[(rodk::R_FX + a) * R + r] = T(h.fend[3 * r + a]);
            rodp[(rodk::R_CX + a) * R + r] = T(h.camp[3 * r + a]);
            rodp[(rodk::R_T0X + a) * R + r] = T(h.pos[3 * (nd + n) + a] - b->origin[3 * r + a]);
        }
        freq[r] = h.cfreq[r];
        phase[r] = h.cphase[r];
        flags[r] = (h.bc0[r] ? rodk::FLAG_CLAMP0 : 0) | (h.bc1[r] ? rodk::FLAG_CLAMP1 : 0)
                 | ((h.has_c && (h.camp[3 * r] != 0 || h.camp[3 * r + 1] != 0 || h.camp[3 * r + 2] != 0))
                        ? rodk::FLAG_COUPLE : 0);
        e += n;
        v += n - 1;
        nd += n + 1;
    }
    // ---- integer tables
    std::vector<int32_t> ints((size_t)2 * NS + 4 * R, 0);
    std::copy(b->slot_rod.begin(), b->slot_rod.end(), ints.begin());
    std::copy(b->slot_idx.begin(), b->slot_idx.end(), ints.begin() + NS);
    std::copy(h.n.begin(), h.n.end(), ints.begin() + 2 * NS);
    std::copy(flags.begin(), flags.end(), ints.begin() + 2 * NS + R);
    std::copy(b->rod_slot.begin(), b->rod_slot.end(), ints.begin() + 2 * NS + 2 * R);
    // ---- device allocations
    const size_t es = sizeof(T);
    HIPCHK(hipMalloc(&b->d_state, (size_t)rodk::N_STATE * NS * es));
    HIPCHK(hipMalloc(&b->d_param, (size_t)rodk::N_PARAM * NS * es));
    HIPCHK(hipMalloc(&b->d_tail, (size_t)rodk::N_TAIL * R * es));
    HIPCHK(hipMalloc(&b->d_rodp, (size_t)rodk::N_RODP * R * es));
    HIPCHK(hipMalloc((void **)&b->d_freq, (size_t)R * sizeof(double)));
    HIPCHK(hipMalloc((void **)&b->d_phase, (size_t)R * sizeof(double)));
    HIPCHK(hipMalloc((void **)&b->d_energy, (size_t)5 * R * sizeof(double)));
    HIPCHK(hipMalloc((void **)&b->d_ints, ints.size() * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&b->d_step, sizeof(int64_t)));
    HIPCHK(hipMemcpy(b->d_param, param.data(), param.size() * es, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_rodp, rodp.data(), rodp.size() * es, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_freq, freq.data(), R * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_phase, phase.data(), R * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_ints, ints.data(), ints.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    const int64_t zero = 0;
    HIPCHK(hipMemcpy(b->d_step, &zero, sizeof(int64_t), hipMemcpyHostToDevice));
    if (b->magnetic) {
        // magnetization times rest length per slot (zero on padding lanes)
        std::vector<T> mag((size_t)3 * NS, T(0));
        int64_t ee = 0;
        for (int r = 0; r < R; ++r) {
            for (int i = 0; i < h.n[r]; ++i)
                for (int a = 0; a < 3; ++a)
                    mag[a * NS + b->rod_slot[r] + i] = T(h.mag[3 * (ee + i) + a] * h.lh[ee + i]);
            ee += h.n[r];
        }
        HIPCHK(hipMalloc(&b->d_mag, mag.size() * es));
        HIPCHK(hipMemcpy(b->d_mag, mag.data(), mag.size() * es, hipMemcpyHostToDevice));
    }
    if (b->grav[0] != 0 || b->grav[1] != 0 || b->grav[2] != 0) {
        // creation positions relative to the rod origin, for the work of gravity
        const int64_t NT = NS + R;
        std::vector<double> r0((size_t)3 * NT, 0.0);
        int64_t nn = 0;
        for (int r = 0; r < R; ++r) {
            for (int j = 0; j <= h.n[r]; ++j) {
                const int64_t col = j < h.n[r] ? b->rod_slot[r] + j : NS + r;
                for (int a = 0; a < 3; ++a) r0[a * NT + col] = h.pos[3 * (nn + j) + a] - b->origin[3 * r + a];
            }
            nn += h.n[r] + 1;
        }
        HIPCHK(hipMalloc((void **)&b->d_grav_r0, r0.size() * sizeof(double)));
        HIPCHK(hipMemcpy(b->d_grav_r0, r0.data(), r0.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!h.ck.empty()) {
        // connections: compact indices of the connected nodes per tile (node j < n of
        // rod r is column 0 of slot rod_slot[r] + j, node n column 1 of the rod's
        // last slot), CSR over them in connection order, spring parameters, and
        // each rod's origin relative to the first rod of its tile
        const int TL = 64 * b->waves;
        const int C = (int)h.ck.size();
        auto key_of = [&](int32_t r, int32_t j) -> int64_t {
            const int n = h.n[r];
            return j < n ? 2 * ((int64_t)b->rod_slot[r] + j) : 2 * ((int64_t)b->rod_slot[r] + n - 1) + 1;
        };
        std::vector<int64_t> keys;
        keys.reserve(2 * C);
        for (int c = 0; c < C; ++c)
            for (int end = 0; end < 2; ++end) keys.push_back(key_of(h.crod[2 * c + end], h.cnode[2 * c + end]));
        std::vector<int64_t> ukeys(keys);
        std::sort(ukeys.begin(), ukeys.end());
        ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
        std::vector<int32_t> idx((size_t)2 * NS, -1), count(b->n_tiles, 0), tbase(b->n_tiles, 0);
        std::vector<int32_t> gidx(ukeys.size());
        for (size_t u = 0; u < ukeys.size(); ++u) {
            const int64_t slot = ukeys[u] / 2;
            const int tile = (int)(slot / TL);
            idx[(ukeys[u] % 2) * NS + slot] = count[tile]++;
        }
        int32_t total = 0;
        for (int t = 0; t < b->n_tiles; ++t) {
            tbase[t] = total;
            total += count[t];
            b->conn_max_nodes = std::max(b->conn_max_nodes, count[t]);
        }
        auto global_of = [&](int64_t key) {
            const int64_t slot = key / 2;
            return tbase[slot / TL] + idx[(key % 2) * NS + slot];
        };
        std::vector<int32_t> ckey(total);
        for (int64_t key : ukeys) ckey[global_of(key)] = (int32_t)key;
        std::vector<int32_t> off(total + 1, 0), partner(2 * C);
        std::vector<double> par((size_t)3 * 2 * C);
        for (int c = 0; c < C; ++c) {
            ++off[global_of(keys[2 * c]) + 1];
            ++off[global_of(keys[2 * c + 1]) + 1];
        }
        for (int32_t g = 0; g < total; ++g) off[g + 1] += off[g];
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int c = 0; c < C; ++c)
            for (int end = 0; end < 2; ++end) {
                const int64_t me = keys[2 * c + end], other = keys[2 * c + 1 - end];
                if ((me / 2) / TL != (other / 2) / TL)
                    return fail(ROD_EDEVICE, "connection " + std::to_string(c) + " spans two tiles");
                const int32_t e = fill[global_of(me)]++;
                partner[e] = idx[(other % 2) * NS + other / 2];
                par[e] = h.ck[c];
                par[2 * C + e] = h.cc[c];
                par[4 * C + e] = h.crest[c];
            }
        b->n_conn = C;
        HIPCHK(hipMalloc((void **)&b->d_conn_idx, idx.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&b->d_conn_tbase, tbase.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&b->d_conn_off, off.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&b->d_conn_partner, partner.size() * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&b->d_conn_key, std::max<size_t>(ckey.size(), 1) * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&b->d_conn_par, par.size() * sizeof(double)));

        HIPCHK(hipMemcpy(b->d_conn_idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_conn_tbase, tbase.data(), tbase.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_conn_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_conn_partner, partner.data(), partner.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_conn_key, ckey.data(), ckey.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_conn_par, par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if (!h.ck.empty() || b->n_walls > 0 || b->rod_contact) {
        // FP32 node interactions work in the frame of each tile's first rod
        // (small coordinates): rod origins relative to it, and the walls'
        // offsets d - n . (its origin) per tile. FP64 keeps lab-frame node
        // positions, so there the reference is the lab origin.
        const bool rel = sizeof(T) == 4;
        const int TL = 64 * b->waves;
        std::vector<int32_t> first_rod(b->n_tiles, -1);
        for (int r = 0; r < R; ++r) {
            const int tile = b->rod_slot[r] / TL;
            if (first_rod[tile] < 0 || b->rod_slot[r] < b->rod_slot[first_rod[tile]]) first_rod[tile] = r;
        }
        std::vector<double> org((size_t)3 * R, 0.0);
        for (int r = 0; r < R; ++r) {
            const int ref = first_rod[b->rod_slot[r] / TL];
            for (int a = 0; a < 3; ++a)
                org[a * R + r] = rel ? b->origin[3 * r + a] - b->origin[3 * ref + a] : 0.0;
        }
        std::vector<T> woff((size_t)8 * b->n_tiles, T(0));
        for (int t = 0; t < b->n_tiles; ++t)
            for (int w = 0; w < b->n_walls; ++w) {
                const double *o = rel && first_rod[t] >= 0 ? &b->origin[3 * first_rod[t]] : nullptr;
                const double shift = o ? b->walls[w][0] * o[0] + b->walls[w][1] * o[1] + b->walls[w][2] * o[2] : 0.0;
                woff[(size_t)8 * t + w] = T(b->walls[w][3] - shift);
            }
        HIPCHK(hipMalloc(&b->d_wall_off, woff.size() * es));
        HIPCHK(hipMemcpy(b->d_wall_off, woff.data(), woff.size() * es, hipMemcpyHostToDevice));
        HIPCHK(hipMalloc((void **)&b->d_rod_org, org.size() * sizeof(double)));
        HIPCHK(hipMemcpy(b->d_rod_org, org.data(), org.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMalloc((void **)&b->d_rod_rad, (size_t)R * sizeof(double)));
        HIPCHK(hipMemcpy(b->d_rod_rad, h.rad.data(), (size_t)R * sizeof(double), hipMemcpyHostToDevice));
    }
    if (b->muscle) {
        // amplitude times axis and the phase offset phi - q s_k at the Voronoi
        // point of each slot (zero amplitude on a rod's first element and padding)
        std::vector<T> mus((size_t)3 * NS, T(0));
        std::vector<double> ofs((size_t)NS, 0.0);
        int64_t ee = 0, vv = 0;
        for (int r = 0; r < R; ++r) {
            double sk = 0.0;
            for (int i = 0; i + 1 < h.n[r]; ++i) {
                sk += h.lh[ee + i];
                const int64_t sl = b->rod_slot[r] + i + 1;   // Voronoi point i lives on slot i+1
                for (int a = 0; a < 3; ++a) mus[a * NS + sl] = T(h.mamp[vv + i] * h.maxis[3 * r + a]);
                ofs[sl] = h.mphase[r] - h.mwave[r] * sk;
            }
            ee += h.n[r];
            vv += h.n[r] - 1;
        }
        HIPCHK(hipMalloc(&b->d_mus, mus.size() * es));
        HIPCHK(hipMalloc((void **)&b->d_mus_ofs, ofs.size() * sizeof(double)));
        HIPCHK(hipMalloc((void **)&b->d_mus_freq, (size_t)R * sizeof(double)));
        HIPCHK(hipMemcpy(b->d_mus, mus.data(), mus.size() * es, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_mus_ofs, ofs.data(), ofs.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->d_mus_freq, h.mfreq.data(), (size_t)R * sizeof(double), hipMemcpyHostToDevice));
    }
    int rc = upload_state<T>(b, h.pos.data(), h.vel.data(), h.dir.data(), h.om.data());
    if (rc) return rc;
    return ROD_OK;
}

// Device buffers of the contact grid: cells of twice the largest radius (plus
// the Verlet skin); per
// axis enough cells (at least 3) to cover the initial extent of the nodes,
// shrunk along the longest axes while the grid holds more than 4 buckets per
// node (or more than the prefix sum takes); the grid wraps beyond that.
int build_contact_grid(rod_batch *b, const HostInputs &h)
{
    rodk::ContactGrid &g = b->cg;
    g.mode = b->contact_mode;
    g.nid = b->n_slots + b->R;
    g.nn = g.mode == 2 ? b->n_slots : g.nid;
    double rmax = 0, lmax = 0;
    for (double r : h.rad) rmax = std::max(rmax, r);
    for (double l : h.lh) lmax = std::max(lmax, l);
    // mode 2: elements are binned by their midpoints; two touching elements'
    // midpoints are at most (l_a + l_b) / 2 + r_a + r_b apart, so cells hold the
    // longest element stretched by a quarter plus twice the largest radius
    g.cell_len = 1.25 * lmax;
    // Verlet lists unless the skin is negative; 0 picks a fifth of the
    // largest radius (a node may then move a tenth of it between builds)
    g.skin = b->contact_skin >= 0 ? (b->contact_skin > 0 ? b->contact_skin : 0.2 * rmax) : 0.0;
    const double cell = (g.mode == 2 ? g.cell_len + 2.0 * rmax : 2.0 * rmax) + g.skin;
    g.inv_cell = 1.0 / cell;
    g.rmax = rmax;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (size_t j = 0; j < h.pos.size() / 3; ++j)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], h.pos[3 * j + a]);
            hi[a] = std::max(hi[a], h.pos[3 * j + a]);
        }
    int64_t n[3];
    for (int a = 0; a < 3; ++a) {
        g.org[a] = lo[a];
        n[a] = std::max<int64_t>(3, (int64_t)std::ceil((hi[a] - lo[a]) / cell) + 1);
        n[a] = std::min<int64_t>(n[a], rodk::CONTACT_MAX_BUCKETS / 9);
    }
    const int64_t budget = std::min<int64_t>(std::max<int64_t>(4 * g.nn, 27), rodk::CONTACT_MAX_BUCKETS);
    while (n[0] * n[1] * n[2] > budget) {
        const int a = n[0] >= n[1] && n[0] >= n[2] ? 0 : (n[1] >= n[2] ? 1 : 2);
        if (n[a] <= 3) break;
        n[a] = std::max<int64_t>(3, (n[a] * 7) / 8);
    }
    g.gx = (int)n[0];
    g.gy = (int)n[1];
    g.gz = (int)n[2];
    const int64_t nb = n[0] * n[1] * n[2], nc = (nb + 1023) / 1024;
    if (nb > rodk::CONTACT_MAX_BUCKETS) return fail(ROD_EUNSUPPORTED, "contact grid too large");
    HIPCHK(hipMalloc((void **)&g.count, nb * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&g.start, (nb + 1) * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&g.chunk, nc * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&g.bucket, g.nn * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&g.rank, g.nn * sizeof(int32_t)));
    HIPCHK(hipMalloc((void **)&g.sid, g.nn * sizeof(int32_t)));
    if (g.mode == 2) {
        HIPCHK(hipMalloc((void **)&g.sca, g.nn * sizeof(double4)));
        HIPCHK(hipMalloc((void **)&g.scb, g.nn * sizeof(double4)));
        HIPCHK(hipMalloc((void **)&g.sva, g.nn * sizeof(double4)));
        HIPCHK(hipMalloc((void **)&g.svb, g.nn * sizeof(double4)));
        HIPCHK(hipMalloc((void **)&g.fseg, 6 * g.nn * sizeof(double)));
        // the elements of its own rod each element may touch: j > i from
        // next[i] on, where the rest lengths strictly between them, summed in
        // increasing order, reach the diameter; j < i up to prev[i], the last
        // j with next[j] <= i (the sums only grow as j moves down, even rounded:
        // a rounded sum of positive terms is monotone in each term)
        const size_t NS = (size_t)b->n_slots;
        std::vector<int32_t> pairs(2 * NS, 0);
        int64_t e = 0;
        for (int r = 0; r < b->R; ++r) {
            const int n = h.n[r];
            const int64_t s0 = b->rod_slot[r];
            for (int i = 0; i < n; ++i) {
                int j = i + 2;
                double gap = j - 1 < n ? h.lh[e + i + 1] : 0.0;
                while (j < n && !(gap >= 2.0 * h.rad[r])) {
                    gap += h.lh[e + j];
                    ++j;
                }
                pairs[s0 + i] = std::min(j, n);
            }
            // next[] does not decrease along the rod, so prev[] follows it
            int prev = -1;
            for (int i = 0; i < n; ++i) {
                while (prev + 1 < n && pairs[s0 + prev + 1] <= i) ++prev;
                pairs[NS + s0 + i] = prev;
            }
            e += n;
        }
        int32_t *d_pairs = nullptr;
        HIPCHK(hipMalloc((void **)&d_pairs, pairs.size() * sizeof(int32_t)));
        g.self_pairs = d_pairs;
        HIPCHK(hipMemcpy(d_pairs, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        // a group of screening records more than the elements: the force pass
        // reads whole groups and masks the records past a range's end
        HIPCHK(hipMalloc((void **)&g.cull, 2 * (g.nn + rodk::CONTACT_PAD) * sizeof(float4)));
    } else {
        // a group of records more than the nodes: the force pass reads whole
        // groups and masks the records past a range's end
        HIPCHK(hipMalloc((void **)&g.spr, (g.nn + rodk::CONTACT_PAD) * sizeof(double4)));
        HIPCHK(hipMalloc((void **)&g.svr, g.nn * sizeof(double4)));
    }
    if (g.skin > 0) {
        // Verlet lists: per item (node, or element slot) its count and entries
        HIPCHK(hipMalloc((void **)&g.lcount, g.nn * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&g.lid, (size_t)rodk::CONTACT_LIST_CAP * g.nn * sizeof(int32_t)));
        HIPCHK(hipMalloc((void **)&g.xb, 3 * g.nid * sizeof(double)));
        HIPCHK(hipMalloc((void **)&g.vflag, rodk::CONTACT_VFLAGS * sizeof(int32_t)));
        // no build yet (NaN positions: the first pass builds)
        const std::vector<double> nan3(3 * g.nid, std::nan(""));
        HIPCHK(hipMemcpy(g.xb, nan3.data(), nan3.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemset(g.lcount, 0, g.nn * sizeof(int32_t)));
        // every entry names a valid item (the list pass reads entries past a count)
        HIPCHK(hipMemset(g.lid, 0, (size_t)rodk::CONTACT_LIST_CAP * g.nn * sizeof(int32_t)));
        HIPCHK(hipMemset(g.vflag, 0, rodk::CONTACT_VFLAGS * sizeof(int32_t)));
        if (g.mode == 2) {
            HIPCHK(hipMalloc((void **)&g.srec, 4 * g.nn * sizeof(double4)));
            HIPCHK(hipMemset(g.srec, 0, 4 * g.nn * sizeof(double4)));
        } else {
            HIPCHK(hipMalloc((void **)&g.rec, 2 * g.nid * sizeof(double4)));
            // padding ids keep rod -1 (the pack kernel writes real nodes only)
            const std::vector<double4> pad(2 * g.nid, make_double4(0.0, 0.0, 0.0, -1.0));
            HIPCHK(hipMemcpy(g.rec, pad.data(), pad.size() * sizeof(double4), hipMemcpyHostToDevice));
            if (b->precision == ROD_F64) {   // FP32 records come from the positions kernel, all of them
                HIPCHK(hipMalloc((void **)&g.need, g.nid));
                HIPCHK(hipMemset(g.need, 0, g.nid));
            }
        }
    }
    HIPCHK(hipMalloc((void **)&g.force, 3 * g.nid * sizeof(double)));
    HIPCHK(hipMalloc((void **)&g.pot, g.nid * sizeof(double)));
    // counts start at zero; each pass clears them as it reads them
    HIPCHK(hipMemset(g.count, 0, nb * sizeof(int32_t)));
    HIPCHK(hipMemset(g.force, 0, 3 * g.nid * sizeof(double)));
    HIPCHK(hipMemset(g.pot, 0, g.nid * sizeof(double)));
    if (b->precision == ROD_F32) {
        // FP32 positions are summed from the rod origins, edges and anchors
        std::vector<double> org((size_t)3 * b->R);
        for (int r = 0; r < b->R; ++r)
            for (int a = 0; a < 3; ++a) org[(size_t)a * b->R + r] = b->origin[3 * r + a];
        double *d_org = nullptr;
        HIPCHK(hipMalloc((void **)&d_org, org.size() * sizeof(double)));
        g.origin = d_org;
        HIPCHK(hipMemcpy(d_org, org.data(), org.size() * sizeof(double), hipMemcpyHostToDevice));
        if (!g.rec) HIPCHK(hipMalloc((void **)&g.xabs, 3 * g.nid * sizeof(double)));   // else in the records
    }
    HIPCHK(hipDeviceSynchronize());
    return ROD_OK;
}

void free_graphs(rod_batch *b)
{
    for (auto &kv : b->graphs) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    b->graphs.clear();
}

int enqueue_steps(rod_batch *b, int64_t n_steps, hipStream_t s)
{
    const int64_t S = b->substeps > 0 ? b->substeps : n_steps;
    for (int64_t done = 0; done < n_steps; done += S) {
        const int n_sub = (int)std::min<int64_t>(S, n_steps - done);
        if (b->rod_contact) {
            // contact forces at the positions after the coming half drift
            hipError_t e = b->precision == ROD_F32 ? rodk::launch_contact(b->b32, b->cg, 0.5 * b->dt, s)
                                                   : rodk::launch_contact(b->b64, b->cg, 0.5 * b->dt, s);
            if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("contact launch: ") + hipGetErrorString(e));
        }
        hipError_t e = b->precision == ROD_F32 ? rodk::launch_step(b->b32, b->waves, n_sub, b->grid, s)
                                               : rodk::launch_step(b->b64, b->waves, n_sub, b->grid, s);
        if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
        // with Verlet lists the pass's closing kernel advances the step counter
        e = b->cg.vflag ? rodk::launch_contact_finish(b->cg, b->d_step, n_sub, s)
                        : rodk::launch_advance(b->d_step, n_sub, s);
        if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("advance launch: ") + hipGetErrorString(e));
    }
    return ROD_OK;
}

int check_flags(rod_batch *b, hipStream_t s, std::vector<int32_t> *out = nullptr)
{
    std::vector<int32_t> f(b->R);
    int32_t *dflags = b->d_ints + 2 * b->n_slots + 3 * b->R;
    HIPCHK(hipMemcpyAsync(f.data(), dflags, b->R * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (out) *out = f;
    for (int r = 0; r < b->R; ++r)
        if (f[r] & ROD_FLAG_NONFINITE) return fail(ROD_ENONFINITE, "rod " + std::to_string(r) + " has a non-finite state");
    return ROD_OK;
}

template <typename T>
int download_state(rod_batch *b, hipStream_t s, double *pos, double *vel, double *dir, double *om)
{
    constexpr bool EDGE = sizeof(T) == 4;
    const int64_t NS = b->n_slots;
    const int R = b->R;
    std::vector<T> state((size_t)rodk::N_STATE * NS), tail((size_t)rodk::N_TAIL * R);
    HIPCHK(hipMemcpyAsync(state.data(), b->d_state, state.size() * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(tail.data(), b->d_tail, tail.size() * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t e = 0, nd = 0;
    for (int r = 0; r < R; ++r) {
        const int n = b->n[r];
        const double *o = &b->origin[3 * r];
        double x[3];
        if (EDGE)   // node 0, then accumulate the edges in FP64
            for (int a = 0; a < 3; ++a) x[a] = (double)tail[(rodk::TRX + a) * R + r] + o[a];
        for (int i = 0; i < n; ++i) {
            const int64_t sl = b->rod_slot[r] + i;
            for (int a = 0; a < 3; ++a) {
                if (pos) {
                    if (EDGE) {
                        pos[3 * (nd + i) + a] = x[a];
                        x[a] += (double)state[(rodk::RX + a) * NS + sl];
                    } else {
                        pos[3 * (nd + i) + a] = (double)state[(rodk::RX + a) * NS + sl] + o[a];
                    }
                }
                if (vel) vel[3 * (nd + i) + a] = (double)state[(rodk::VX + a) * NS + sl];
                if (om) om[3 * (e + i) + a] = (double)state[(rodk::WX + a) * NS + sl];
            }
            if (dir)
                for (int k = 0; k < 9; ++k) dir[9 * (e + i) + k] = (double)state[(rodk::Q00 + k) * NS + sl];
        }
        for (int a = 0; a < 3; ++a) {
            if (pos) pos[3 * (nd + n) + a] = EDGE ? x[a] : (double)tail[(rodk::TRX + a) * R + r] + o[a];
            if (vel) vel[3 * (nd + n) + a] = (double)tail[(rodk::TVX + a) * R + r];
        }
        e += n;
        nd += n + 1;
    }
    return ROD_OK;
}

}  // namespace

int rodk::batch_view(const rod_batch *b, BatchView *v)
{
    if (!b || !v) return fail(ROD_EINVAL, "batch is NULL");
    v->precision = b->precision;
    v->waves = b->waves;
    v->extended = b->ext;
    v->n_rods = b->R;
    v->n_elems = b->Ne;
    v->n_slots = b->n_slots;
    v->n = b->n.data();
    v->rod_slot = b->rod_slot.data();
    v->youngs = b->E.data();
    v->shear_modulus = b->G.data();
    v->density = b->rho.data();
    v->radius = b->rad.data();
    v->shear_coeff = b->ac.data();
    v->couple_amp = b->camp.data();
    v->couple_freq = b->cfreq.data();
    v->couple_phase = b->cphase.data();
    v->bc_start = b->bc0.data();
    v->bc_end = b->bc1.data();
    v->dt = b->dt;
    v->time = b->t0 + (double)b->steps * b->dt;
    v->f32 = b->b32;
    v->state_bytes = (size_t)rodk::N_STATE * b->n_slots * elem_bytes(b);
    v->tail_bytes = (size_t)rodk::N_TAIL * b->R * elem_bytes(b);
    return ROD_OK;
}

int rodk::batch_advance_clock(rod_batch *b, int64_t n, hipStream_t s)
{
    hipError_t e = rodk::launch_advance(b->d_step, n, s);
    if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("advance: ") + hipGetErrorString(e));
    b->steps += n;
    return ROD_OK;
}

int rodk::batch_step_masked(rod_batch *b, int64_t n, const int32_t *active, const int32_t *tile_list, int n_list,
                            hipStream_t s)
{
    if (n_list <= 0 || !tile_list) return fail(ROD_EINVAL, "masked step needs a non-empty tile list");
    b->b32.active = b->b64.active = active;
    b->b32.tile_list = b->b64.tile_list = tile_list;
    b->b32.n_list = b->b64.n_list = n_list;
    const int grid = b->grid;
    b->grid = std::min(grid, n_list);
    const int rc = enqueue_steps(b, n, s);
    b->grid = grid;
    b->b32.active = b->b64.active = nullptr;
    b->b32.tile_list = b->b64.tile_list = nullptr;
    b->b32.n_list = b->b64.n_list = 0;
    if (rc) return rc;
    b->steps += n;
    return ROD_OK;
}

int rodk::batch_set_time(rod_batch *b, double t, hipStream_t s)
{
    hipError_t e = rodk::launch_set_step(b->d_step, 0, s);
    if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("set step: ") + hipGetErrorString(e));
    b->t0 = t;
    b->steps = 0;
    fill_dev(b->b64, b);
    fill_dev(b->b32, b);
    free_graphs(b);
    b->use_graphs = false;
    return ROD_OK;
}

namespace {

// Time every candidate (tile width x substeps per launch) on scratch batches
// of the same rods and return the fastest in `best` (autotune cleared).
int autotune(const rod_batch_desc *d, std::vector<rod_tune_trial> &log, rod_batch_desc &best)
{
    constexpr int TRIAL_STEPS = 1000;
    const std::vector<int> widths = d->tile_waves ? std::vector<int>{d->tile_waves} : std::vector<int>{1, 2, 4, 8};
    const std::vector<int> subs = d->substeps  ? std::vector<int>{d->substeps}
                                : d->rod_contact ? std::vector<int>{1}
                                                 : std::vector<int>{50, 200, 1000};
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    };
    hipError_t he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        release();
        return fail(ROD_EDEVICE, std::string("autotune set-up: ") + hipGetErrorString(he));
    }
    best = *d;
    best.autotune = 0;
    double best_ns = INFINITY;
    for (int w : widths) {
        rod_batch_desc c = *d;
        c.autotune = 0;
        c.tile_waves = w;
        c.substeps = subs[0];
        rod_batch *tb = nullptr;
        int rc = rod_batch_create(&c, nullptr, &tb);
        if (rc == ROD_EUNSUPPORTED) continue;   // this width cannot hold the longest rod
        if (rc) {
            release();
            return rc;
        }
        tb->use_graphs = false;
        for (int sub : subs) {
            tb->substeps = sub;
            rc = enqueue_steps(tb, sub, st);   // warm-up launch
            if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = fail(ROD_EDEVICE, "autotune: event record");
            if (!rc) rc = enqueue_steps(tb, TRIAL_STEPS, st);
            if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(ROD_EDEVICE, "autotune: event record");
            float ms = 0.f;
            if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(ROD_EDEVICE, "autotune: event timing");
            if (rc) {
                rod_batch_destroy(tb);
                release();
                return rc;
            }
            const double ns = (double)ms * 1e6 / ((double)tb->Ne * TRIAL_STEPS);
            log.push_back(rod_tune_trial{w, sub, ns});
            if (ns < best_ns) {
                best_ns = ns;
                best.tile_waves = w;
                best.substeps = sub;
            }
        }
        rod_batch_destroy(tb);
    }
    release();
    if (log.empty()) return fail(ROD_EUNSUPPORTED, "autotune: no tile width holds the longest rod");
    return ROD_OK;
}

}  // namespace

extern "C" {

const char *rod_last_error(void) { return g_err.c_str(); }

int rod_batch_tuning(const rod_batch *b, rod_tune_trial *trials, int32_t max_trials, int32_t *n_trials)
{
    if (!b || !n_trials || (max_trials > 0 && !trials) || max_trials < 0)
        return fail(ROD_EINVAL, "NULL handle or output, or max_trials < 0");
    const int32_t n = (int32_t)std::min<size_t>(b->tune_log.size(), (size_t)max_trials);
    for (int32_t i = 0; i < n; ++i) trials[i] = b->tune_log[i];
    *n_trials = (int32_t)b->tune_log.size();
    return ROD_OK;
}

int rod_batch_create(const rod_batch_desc *d, void *stream, rod_batch **out)
{
    g_err.clear();
    if (!out) return fail(ROD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(d);
    if (rc) return rc;
    if (d->autotune && (d->tile_waves == 0 || d->substeps == 0)) {
        std::vector<rod_tune_trial> log;
        rod_batch_desc best;
        if ((rc = autotune(d, log, best))) return rc;
        if ((rc = rod_batch_create(&best, stream, out))) return rc;
        (*out)->tune_log = std::move(log);
        return ROD_OK;
    }
    HostInputs h;
    if ((rc = gather_inputs(d, h))) return rc;
    if ((rc = check_values(h))) return rc;
    (void)stream;

    auto *b = new (std::nothrow) rod_batch();
    if (!b) return fail(ROD_ENOMEM, "host allocation failed");
    b->precision = d->precision;
    b->substeps = d->substeps;
    b->R = d->n_rods;
    b->n = h.n;
    b->dt = d->dt;
    b->t0 = d->t0;
    b->use_graphs = std::getenv("ROD_NO_GRAPH") == nullptr;
    const auto groups = connected_groups(b->R, h.crod);
    int nmax = 0;   // the largest group (a rod, or rods joined by connections)
    for (const auto &g : groups) {
        int sz = 0;
        for (int32_t r : g) sz += h.n[r];
        nmax = std::max(nmax, sz);
    }
    for (int r = 0; r < b->R; ++r) b->Ne += h.n[r];
    b->Nn = b->Ne + b->R;
    int waves = d->tile_waves;
    const int need = (nmax + 63) / 64;
    if (waves == 0) {
        waves = 1;
        while (waves < need) waves *= 2;
    }
    if (waves < need) {
        delete b;
        return fail(ROD_EUNSUPPORTED, "tile_waves " + std::to_string(waves) + " cannot hold a rod or connected group of "
                                          + std::to_string(nmax) + " elements");
    }
    b->waves = waves;
    if (nmax > 64 * 8) {
        delete b;
        return fail(ROD_EUNSUPPORTED, "a connected group of " + std::to_string(nmax) + " elements exceeds a tile (512)");
    }
    pack_tiles(h.n, groups, 64 * waves, b->rod_slot, b->n_tiles);
    b->n_slots = (int64_t)b->n_tiles * 64 * waves;
    b->slot_rod.assign(b->n_slots, -1);
    b->slot_idx.assign(b->n_slots, 0);
    for (int r = 0; r < b->R; ++r)
        for (int i = 0; i < h.n[r]; ++i) {
            b->slot_rod[b->rod_slot[r] + i] = r;
            b->slot_idx[b->rod_slot[r] + i] = i;
        }
    // rod origins (FP32 keeps positions relative to the first node)
    b->origin.assign(3 * b->R, 0.0);
    b->bc0 = h.bc0;
    b->bc1 = h.bc1;
    b->E = h.E;
    b->G = h.G;
    b->rho = h.rho;
    b->rad = h.rad;
    b->ac = h.ac;
    b->camp = h.camp;
    b->cfreq = h.cfreq;
    b->cphase = h.cphase;
    b->magnetic = d->magnetization != nullptr;
    if (b->magnetic) {
        for (int k = 0; k < 9; ++k) b->field[k] = d->field[k];
        b->field_freq = d->field_freq;
    }
    b->muscle = d->muscle_amp != nullptr;
    for (int a = 0; a < 3; ++a) b->grav[a] = d->gravity[a];
    b->n_walls = d->n_walls;
    for (int w = 0; w < d->n_walls; ++w)
        for (int k = 0; k < 4; ++k) b->walls[w][k] = d->walls[4 * w + k];
    b->wall_k = d->wall_k;
    b->wall_c = d->wall_c;
    b->wall_mu = d->wall_mu;
    b->wall_vslip = d->wall_vslip;
    b->rod_contact = d->rod_contact != 0;
    b->contact_mode = d->rod_contact;
    b->contact_skin = d->contact_skin;
    if (b->rod_contact) b->substeps = 1;   // a contact pass before every step
    b->ext = b->magnetic || b->muscle || d->gravity[0] != 0 || d->gravity[1] != 0 || d->gravity[2] != 0
           || d->n_connections > 0 || d->n_walls > 0 || b->rod_contact;
    b->clamp_r0.assign(3 * b->R, 0.0);
    b->clamp_rn.assign(3 * b->R, 0.0);
    b->clamp_q0.assign(9 * b->R, 0.0);
    b->clamp_qn.assign(9 * b->R, 0.0);
    {
        int64_t e = 0, nd = 0;
        for (int r = 0; r < b->R; ++r) {
            const int n = h.n[r];
            for (int a = 0; a < 3; ++a) {
                if (b->precision == ROD_F32) b->origin[3 * r + a] = h.pos[3 * nd + a];
                b->clamp_r0[3 * r + a] = h.pos[3 * nd + a];
                b->clamp_rn[3 * r + a] = h.pos[3 * (nd + n) + a];
            }
            for (int k = 0; k < 9; ++k) {
                b->clamp_q0[9 * r + k] = h.dir[9 * e + k];
                b->clamp_qn[9 * r + k] = h.dir[9 * (e + n - 1) + k];
            }
            e += n;
            nd += n + 1;
        }
    }
    rc = b->precision == ROD_F32 ? build_device<float>(b, h) : build_device<double>(b, h);
    if (!rc && b->rod_contact) rc = build_contact_grid(b, h);
    if (rc) {
        rod_batch_destroy(b);
        return rc;
    }
    fill_dev(b->b64, b);
    fill_dev(b->b32, b);
    b->grid = b->n_tiles;
    {
        // the kernel this batch runs must fit the workgroup's LDS
        const int kind = !b->ext ? 0
                       : (b->n_walls > 0 || b->rod_contact) ? (b->n_conn > 0 ? 3 : 4) : b->n_conn > 0 ? 2 : 1;
        int dev = 0, limit = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) limit = 65536;
        const size_t need = rodk::step_lds_bytes(b->precision == ROD_F32, b->waves, kind, b->conn_max_nodes);
        if (need > (size_t)limit) {
            rod_batch_destroy(b);
            return fail(ROD_EUNSUPPORTED, "tiles of " + std::to_string(waves) + " waves need " + std::to_string(need)
                                              + " bytes of LDS for this batch (the device allows "
                                              + std::to_string(limit) + "); use narrower tiles");
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        rod_batch_destroy(b);
        return fail(ROD_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    const double dts = stability_dt(h, d->field, d->n_walls > 0 ? d->wall_k : 0.0, b->rod_contact ? d->wall_k : 0.0);
    if (d->dt > dts) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "warning: dt %.3g exceeds the explicit stability estimate %.3g", d->dt, dts);
        g_err = buf;
    }
    *out = b;
    return ROD_OK;
}

int rod_step(rod_batch *b, int64_t n_steps, void *stream)
{
    if (!b) return fail(ROD_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(ROD_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return ROD_OK;
    hipStream_t s = (hipStream_t)stream;
    if (!b->use_graphs) {
        int rc = enqueue_steps(b, n_steps, s);
        if (rc) return rc;
        b->steps += n_steps;
        return ROD_OK;
    }
    // A graph holds at most 64 step launches (a multiple of the substeps per
    // launch, so the launches split the steps exactly as one long sequence
    // would): rod_step(n) replays it as often as it fits, then a graph of the
    // rest.  One-step launches (rod contact) would otherwise put some ten
    // kernel nodes per step into one graph.
    const int64_t chunk = b->substeps > 0 ? std::min<int64_t>(n_steps, 64 * (int64_t)b->substeps) : n_steps;
    auto graph_of = [&](int64_t steps, hipGraphExec_t &x) -> int {
        auto it = b->graphs.find(steps);
        if (it == b->graphs.end()) {
            if (b->graphs.size() >= 16) free_graphs(b);
            HIPCHK(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_steps(b, steps, b->capture_stream);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(b->capture_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return fail(ROD_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
            hipGraphExec_t e = nullptr;
            ec = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
            if (ec != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(ROD_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
            }
            it = b->graphs.emplace(steps, std::make_pair(g, e)).first;
        }
        x = it->second.second;
        return ROD_OK;
    };
    const int64_t reps = n_steps / chunk, rest = n_steps % chunk;
    hipGraphExec_t xc = nullptr, xr = nullptr;
    int rc = graph_of(chunk, xc);
    if (!rc && rest) rc = graph_of(rest, xr);
    if (rc) return rc;
    if (rest && !b->graphs.count(chunk)) {
        // capturing the rest evicted the chunk's graph (cache full): capture it again
        rc = graph_of(chunk, xc);
        if (rc) return rc;
    }
    for (int64_t k = 0; k < reps; ++k) HIPCHK(hipGraphLaunch(xc, s));
    if (rest) HIPCHK(hipGraphLaunch(xr, s));
    b->steps += n_steps;
    return ROD_OK;
}

int rod_energy(rod_batch *b, double *out, void *stream)
{
    if (!b || !out) return fail(ROD_EINVAL, "handle or out is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (b->rod_contact) {
        // the pairs' potentials at the current positions
        hipError_t e = b->precision == ROD_F32 ? rodk::launch_contact(b->b32, b->cg, 0.0, s)
                                               : rodk::launch_contact(b->b64, b->cg, 0.0, s);
        if (e == hipSuccess && b->cg.vflag) e = rodk::launch_contact_finish(b->cg, nullptr, 0, s);
        if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("contact launch: ") + hipGetErrorString(e));
    }
    hipError_t e = b->precision == ROD_F32 ? rodk::launch_energy(b->b32, b->d_energy, s)
                                           : rodk::launch_energy(b->b64, b->d_energy, s);
    if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("energy launch: ") + hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(out, b->d_energy, (size_t)5 * b->R * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return check_flags(b, s);
}

int rod_energy_noalloc(rod_batch *b, double *out, void *stream)
{
    if (!b || !out) return fail(ROD_EINVAL, "handle or out is NULL");
    if (b->R > rodk::NOALLOC_MAX_RODS)
        return fail(ROD_EINVAL, "rod_energy_noalloc serves at most " + std::to_string(rodk::NOALLOC_MAX_RODS)
                                    + " rods; this batch has " + std::to_string(b->R) + " (use rod_energy)");
    double *energies = nullptr;
    int32_t *first = nullptr;
    int rc = rodk::noalloc_scratch(&energies, &first);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (b->rod_contact) {
        // the pairs' potentials at the current positions (the batch's own grid buffers)
        hipError_t e = b->precision == ROD_F32 ? rodk::launch_contact(b->b32, b->cg, 0.0, s)
                                               : rodk::launch_contact(b->b64, b->cg, 0.0, s);
        if (e == hipSuccess && b->cg.vflag) e = rodk::launch_contact_finish(b->cg, nullptr, 0, s);
        if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("contact launch: ") + hipGetErrorString(e));
    }
    hipError_t e = b->precision == ROD_F32 ? rodk::launch_energy(b->b32, energies, s)
                                           : rodk::launch_energy(b->b64, energies, s);
    if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("energy launch: ") + hipGetErrorString(e));
    const int32_t *dflags = b->d_ints + 2 * b->n_slots + 3 * b->R;
    e = rodk::launch_first_flagged(dflags, b->R, first, s);
    if (e != hipSuccess) return fail(ROD_EDEVICE, std::string("flag launch: ") + hipGetErrorString(e));
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(out, energies, (size_t)5 * b->R * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&bad, first, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad < b->R) return fail(ROD_ENONFINITE, "rod " + std::to_string(bad) + " has a non-finite state");
    return ROD_OK;
}

int rod_get_state(rod_batch *b, double *pos, double *vel, double *dir, double *om, double *t, void *stream)
{
    if (!b) return fail(ROD_EINVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    int rc = b->precision == ROD_F32 ? download_state<float>(b, s, pos, vel, dir, om)
                                     : download_state<double>(b, s, pos, vel, dir, om);
    if (rc) return rc;
    if (t) *t = b->t0 + (double)b->steps * b->dt;
    return check_flags(b, s);
}

int rod_set_state(rod_batch *b, const double *pos, const double *vel, const double *dir, const double *om,
                  double t, void *stream)
{
    if (!b) return fail(ROD_EINVAL, "handle is NULL");
    if (!std::isfinite(t)) return fail(ROD_EINVAL, "t must be finite");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    // fields left NULL keep their current values
    std::vector<double> cp(3 * b->Nn), cv(3 * b->Nn), cd(9 * b->Ne), co(3 * b->Ne);
    int rc = b->precision == ROD_F32 ? download_state<float>(b, s, cp.data(), cv.data(), cd.data(), co.data())
                                     : download_state<double>(b, s, cp.data(), cv.data(), cd.data(), co.data());
    if (rc) return rc;
    const double *P = pos ? pos : cp.data(), *V = vel ? vel : cv.data();
    const double *D = dir ? dir : cd.data(), *O = om ? om : co.data();
    rc = b->precision == ROD_F32 ? upload_state<float>(b, P, V, D, O) : upload_state<double>(b, P, V, D, O);
    if (rc) return rc;
    int32_t *dflags = b->d_ints + 2 * b->n_slots + 3 * b->R;
    HIPCHK(hipMemset(dflags, 0, b->R * sizeof(int32_t)));
    const int64_t zero = 0;
    HIPCHK(hipMemcpy(b->d_step, &zero, sizeof(int64_t), hipMemcpyHostToDevice));
    b->t0 = t;
    b->steps = 0;
    fill_dev(b->b64, b);
    fill_dev(b->b32, b);
    free_graphs(b);   // captured launches hold the old t0
    return ROD_OK;
}

int rod_get_flags(rod_batch *b, int32_t *nonfinite, void *stream)
{
    if (!b || !nonfinite) return fail(ROD_EINVAL, "handle or out is NULL");
    std::vector<int32_t> f;
    int rc = check_flags(b, (hipStream_t)stream, &f);
    if (rc && rc != ROD_ENONFINITE) return rc;
    std::memcpy(nonfinite, f.data(), b->R * sizeof(int32_t));
    return ROD_OK;
}

int rod_batch_info(const rod_batch *b, int64_t *info)
{
    if (!b || !info) return fail(ROD_EINVAL, "handle or info is NULL");
    info[0] = b->R;
    info[1] = b->Ne;
    info[2] = b->n_tiles;
    info[3] = b->waves;
    info[4] = b->substeps;
    info[5] = b->precision;
    info[6] = b->n_slots;
    info[7] = b->steps;
    return ROD_OK;
}

int rod_contact_stats(rod_batch *b, int64_t *out, void *stream)
{
    if (!b || !out) return fail(ROD_EINVAL, "handle or out is NULL");
    for (int k = 0; k < 5; ++k) out[k] = 0;
    if (!b->cg.vflag) return ROD_OK;
    hipStream_t s = (hipStream_t)stream;
    int32_t f[rodk::CONTACT_VFLAGS];
    HIPCHK(hipMemcpyAsync(f, b->cg.vflag, sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out[0] = (uint32_t)f[rodk::VF_PASSES];
    out[1] = (uint32_t)f[rodk::VF_BUILDS];
    out[2] = (uint32_t)f[rodk::VF_FALLBACKS];
    out[3] = f[rodk::VF_MOST];
    out[4] = rodk::CONTACT_LIST_CAP;
    return ROD_OK;
}

void rod_batch_destroy(rod_batch *b)
{
    if (!b) return;
    free_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    (void)hipFree(b->d_state);
    (void)hipFree(b->d_param);
    (void)hipFree(b->cg.count);
    (void)hipFree(b->cg.start);
    (void)hipFree(b->cg.chunk);
    (void)hipFree(b->cg.bucket);
    (void)hipFree(b->cg.rank);
    (void)hipFree(b->cg.spr);
    (void)hipFree(b->cg.svr);
    (void)hipFree(b->cg.sca);
    (void)hipFree(b->cg.scb);
    (void)hipFree(b->cg.sva);
    (void)hipFree(b->cg.svb);
    (void)hipFree(b->cg.fseg);
    (void)hipFree((void *)b->cg.self_pairs);
    (void)hipFree(b->cg.sid);
    (void)hipFree(b->cg.cull);
    (void)hipFree((void *)b->cg.origin);
    (void)hipFree(b->cg.xabs);
    (void)hipFree(b->cg.force);
    (void)hipFree(b->cg.pot);
    (void)hipFree(b->cg.lcount);
    (void)hipFree(b->cg.lid);
    (void)hipFree(b->cg.xb);
    (void)hipFree(b->cg.rec);
    (void)hipFree(b->cg.need);
    (void)hipFree(b->cg.srec);
    (void)hipFree(b->cg.vflag);
    (void)hipFree(b->d_tail);
    (void)hipFree(b->d_rodp);
    (void)hipFree(b->d_mag);
    (void)hipFree(b->d_mus);
    (void)hipFree(b->d_mus_ofs);
    (void)hipFree(b->d_mus_freq);
    (void)hipFree(b->d_grav_r0);
    (void)hipFree(b->d_conn_idx);
    (void)hipFree(b->d_conn_tbase);
    (void)hipFree(b->d_conn_off);
    (void)hipFree(b->d_conn_partner);
    (void)hipFree(b->d_conn_key);
    (void)hipFree(b->d_conn_par);
    (void)hipFree(b->d_rod_org);
    (void)hipFree(b->d_rod_rad);
    (void)hipFree(b->d_wall_off);
    (void)hipFree(b->d_freq);
    (void)hipFree(b->d_phase);
    (void)hipFree(b->d_energy);
    (void)hipFree(b->d_ints);
    (void)hipFree(b->d_step);
    delete b;
}

}  // extern "C"
