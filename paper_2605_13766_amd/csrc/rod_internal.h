// Private declarations shared by the host runtime (rod_lib.cpp) and the HIP
// kernels (rod_kernels.hip) of librod.so.  Not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>

struct rod_batch;
typedef struct rod_batch rod_batch_opaque;

namespace rodk {

// Record the message returned by rod_last_error() for this thread; returns code.
int set_error(int code, const std::string &msg);

// Per-slot state fields.  A slot is one lane of a workgroup tile; slot s of a
// rod holds its node s's position (FP64) or its element s's edge vector
// r_{s+1} - r_s (FP32) in RX..RZ, its node s's velocity and its element s's
// frame and angular velocity.  The per-rod tail arrays hold node n's position
// (FP64) or node 0's position relative to the rod origin (FP32), and node n's
// velocity.
enum StateField {
    RX, RY, RZ, VX, VY, VZ,
    Q00, Q01, Q02, Q10, Q11, Q12, Q20, Q21, Q22,
    WX, WY, WZ,
    N_STATE
};

// Per-slot constants, derived in FP64 on the host.  Node quantities belong to
// the slot's node, element quantities to its element, Voronoi quantities to
// the Voronoi point between the previous element and the slot's element
// (placeholders with zero stiffness on a rod's first slot).
enum ParamField {
    P_INV_M,    // node: 1 / lumped mass
    P_LH,       // element: rest length
    P_INV_LH,   // element: 1 / rest length
    P_J1,       // element: rho I1 lh (= rho I2 lh; rho I3 lh = 2 P_J1)
    P_S1,       // element: alpha_c G A (= S22)
    P_S3,       // element: E A
    P_DH,       // Voronoi: rest length (lh_k + lh_{k+1}) / 2
    P_INV_DH,   // Voronoi: 1 / P_DH
    P_B1,       // Voronoi: bending stiffness E I1 (= E I2), rest-length weighted
    P_B3,       // Voronoi: twist stiffness G I3, rest-length weighted
    P_K0X, P_K0Y, P_K0Z,   // Voronoi: rest curvature
    N_PARAM
};

// Per-rod tail: node n's position (FP64) or node 0's relative to the rod
// origin (FP32, the anchor), and node n's velocity.
enum TailField { TRX, TRY, TRZ, TVX, TVY, TVZ, N_TAIL };

// Per-rod constants in the state precision.
enum RodParam {
    R_GAMMA,                  // linear damping
    R_INV_M_TAIL,             // 1 / mass of node n
    R_FX, R_FY, R_FZ,         // constant force on node n
    R_CX, R_CY, R_CZ,         // couple amplitude per unit length (material frame)
    R_T0X, R_T0Y, R_T0Z,      // position of node n at creation (work of the end force)
    N_RODP
};

enum RodFlags { FLAG_CLAMP0 = 1, FLAG_CLAMP1 = 2, FLAG_COUPLE = 4 };

constexpr int DEV_MAX_WALLS = 8;   // planar walls a batch may hold

template <typename T>
struct DevBatch {
    T *state;              // [N_STATE][n_slots]
    T *param;              // [N_PARAM][n_slots]
    T *tail;               // [N_TAIL][n_rods]
    T *rodp;               // [N_RODP][n_rods]
    double *rod_freq;      // [n_rods] Hz
    double *rod_phase;     // [n_rods] rad
    int32_t *slot_rod;     // [n_slots] rod of the slot, -1 for padding
    int32_t *slot_idx;     // [n_slots] element index within the rod
    int32_t *rod_n;        // [n_rods] elements
    int32_t *rod_flags;    // [n_rods] RodFlags
    int32_t *rod_slot;     // [n_rods] slot of element 0
    int32_t *nonfinite;    // [n_rods] set to 1 when the state stops being finite
    int64_t *step;         // global step counter (device)
    const int32_t *active; // [n_rods] or NULL: rods with active[r] == 0 keep their state
    const int32_t *tile_list;  // [n_list] or NULL: visit only these tiles (all tiles when NULL)
    int n_list;
    int64_t n_slots;
    int32_t n_rods;
    int32_t n_tiles;
    double dt;
    double t0;
    // magnetic couple: [3][n_slots] magnetization times rest length (material
    // frame), NULL for batches without one; the lab field
    // b(t) = field[0:3] + field[3:6] cos(2 pi field_freq t) + field[6:9] sin(...)
    const T *mag;
    T field[9];
    double field_freq;
    double field_ds, field_dc;   // sin, cos of 2 pi field_freq dt
    // extended step (magnetic couple, gravity, muscle torques): when false the
    // plain kernel runs and the fields below are unused
    bool ext;
    T grav[3];                 // gravity, lab frame
    const T *mus;              // [3][n_slots] muscle amplitude x axis at the slot's Voronoi point, or NULL
    const double *mus_ofs;     // [n_slots] phi - q s_k
    const double *mus_freq;    // [n_rods] Hz
    // creation positions relative to the rod origin (work of gravity), FP64:
    // [3][n_slots + n_rods], the slot's node, then each rod's node n; NULL
    // without gravity
    const double *grav_r0;
    // connections (NULL conn_idx: none).  A connected node has a compact index
    // within its tile; the kernel keeps its position and velocity in a
    // dynamic-LDS table of conn_nodes rows per tile.
    const int32_t *conn_idx;       // [2][n_slots]: the slot's node i, and node n on a rod's last slot; -1: none
    const int32_t *conn_tbase;     // [n_tiles] first global compact index of each tile
    const int32_t *conn_off;       // [total + 1] CSR offsets over global compact indices
    const int32_t *conn_partner;   // [2C] partner's compact index within the tile
    const int32_t *conn_key;       // [total] slot * 2 + (0: node i, 1: node n) of each compact index
    const double *conn_par;        // [3][2C] k, c, rest
    const double *rod_org;         // [3][n_rods] rod origin relative to its tile's first rod (connections or walls)
    const double *rod_rad;         // [n_rods] rod radius (connections or walls)
    const T *wall_off;             // [n_tiles][8] wall offsets d in each tile's frame
    int conn_nodes;                // table rows per tile
    int64_t conn_entries;          // 2C
    // planar walls: n.x = d with the solid on the side n.x < d (d in the lab
    // frame; the kernels use wall_off)
    int n_walls;
    T wall[DEV_MAX_WALLS][4];
    T wall_k, wall_c, wall_mu, wall_vslip;
    // rod-rod contact (one step per launch): the contact force
    // on every node for the coming kick, [3][n_slots + n_rods] by node id (the
    // slot's node i, then each rod's node n), and each node's share of the
    // pairs' penalty potential [n_slots + n_rods] (energy passes); NULL
    // without contact
    const double *cforce;
    const double *cpot;
};

// The contact grid of a batch with rod-rod contact: nodes (mode 1) or element
// midpoints (mode 2) are binned by a wrapped uniform grid of gx x gy x gz
// buckets (cell = twice the largest radius, or 1.25 x the longest rest length
// plus twice the largest radius, so every pair in contact lies in neighbouring
// cells; with at least 3 cells per axis the 27 cells around an item are 27
// different buckets; the counts per axis cover the batch's initial extent,
// within a bucket budget), counted, prefix-summed and put into bucket order;
// each item then sums its contacts over its 27 neighbouring buckets.
struct ContactGrid {
    int mode;          // 1: nodes as spheres; 2: elements as capsules (segments), self-contact included
    int64_t nn;        // items binned: node ids n_slots + n_rods (mode 1), element slots n_slots (mode 2)
    int64_t nid;       // node ids: n_slots + n_rods (the stride of force, pot and xabs)
    int gx, gy, gz;    // cells per axis of the wrapped grid, each >= 3
    double inv_cell;   // 1 / cell size
    double rmax;       // the largest rod radius
    double org[3];     // grid origin (the initial extent's lower corner)
    int32_t *count;    // [gx gy gz] items per bucket; zero between passes
    int32_t *start;    // [gx gy gz + 1] first sorted position of each bucket
    int32_t *chunk;    // [ceil(gx gy gz / 1024)] chunk totals of the prefix sum
    int32_t *bucket;   // [nn] an item's bucket
    int32_t *rank;     // [nn] its rank within the bucket, -1 for padding slots
    double4 *spr;      // mode 1: [nn + CONTACT_PAD] position and rod (as a double) in bucket order
    double4 *svr;      // mode 1: [nn] velocity and radius in bucket order
    int32_t *sid;      // [nn] item ids (node ids, or element slots) in bucket order
    // mode 2: [2 (nn + CONTACT_PAD)] screening records in bucket order, two float4 per element:
    // its capsule's bounding box (centre relative to org, half extents), rod, element
    float4 *cull;
    double *force;     // [3][nid] contact force by node id
    double *pot;       // [nid] potential share by node id (mode 2: each element's share at its slot)
    const double *origin;   // FP32 batches: [3][n_rods] rod origins
    double *xabs;      // FP32 batches: [3][nid] node positions (summed in FP64) after the drift
    // mode 2: segment records in bucket order, 128 bytes each: (A, radius), (B, rod),
    // (v_A, element), (v_B, unused)
    double4 *sca, *scb, *sva, *svb;
    // [2][n_slots] the elements of its own rod each element may touch: from
    // `next` on and up to `prev` (the rest lengths between them add up to the
    // diameter; next = n and prev = -1 when there are none)
    const int32_t *self_pairs;
    double *fseg;      // [6][nn] each element's force shares of its nodes A and B
    double cell_len;   // mode 2: the longest element the grid allows for (the cell holds it)
    // Verlet lists (skin > 0; cells grow by the skin): each item's partners
    // when the lists were built, by increasing id - mode 1: the nodes of other
    // rods within its radius + rmax + skin; mode 2: the elements it may touch
    // whose segments were within the two radii + skin - rebuilt when a node
    // has moved more than skin / 2 since
    double skin;       // 0: no lists (the grid pass every step)
    int32_t *lcount;   // [nn] partners listed (more than CONTACT_LIST_CAP: the build overflowed)
    int32_t *lid;      // [CONTACT_LIST_CAP][nn] partner ids (every entry a valid item)
    double *xb;        // [3][nid] node positions at the last build (NaN: none yet, or the node was not finite)
    double4 *rec;      // mode 1: [2 nid] per pass: (position after the drift, radius), (velocity, rod) of each id
    uint8_t *need;     // mode 1, FP64: [nid] 1 for the nodes whose records the lists use (the pack writes only those)
    double4 *srec;     // mode 2: [4 nn] per pass: (A, radius), (B, rod), (v_A, element), (v_B, 0) of each element slot
    // [CONTACT_VFLAGS]: this pass builds, this pass's build overflowed; then
    // counters (passes, builds, builds that overflowed, most partners of one
    // item at a build)
    int32_t *vflag;
};
constexpr int64_t CONTACT_PAD = 4;   // sorted records past the last item (a screening group reads past a range)
constexpr int CONTACT_LIST_CAP = 32; // partners a node's Verlet list holds
constexpr int CONTACT_VFLAGS = 8;
enum { VF_REQUEST = 0, VF_OVERFLOW, VF_PASSES, VF_BUILDS, VF_FALLBACKS, VF_MOST };
constexpr int64_t CONTACT_MAX_BUCKETS = 4096 * 1024;   // chunk totals fit one workgroup's prefix sum

// Fill g.force and g.pot for positions advanced by `drift` seconds from the
// state (dt/2 before a step's kick, 0 for energies).
hipError_t launch_contact(const DevBatch<double> &b, const ContactGrid &g, double drift, hipStream_t s);
hipError_t launch_contact(const DevBatch<float> &b, const ContactGrid &g, double drift, hipStream_t s);
// With Verlet lists (g.skin > 0), after every pass and the step kernel that
// follows it: advance *step by n (step may be NULL) and settle the pass's flags.
hipError_t launch_contact_finish(const ContactGrid &g, int64_t *step, int64_t n, hipStream_t s);

// Kernel launchers (rod_kernels.hip).  `waves` is the tile width in wave64s.
hipError_t launch_step(const DevBatch<double> &b, int waves, int n_sub, int grid, hipStream_t s);
hipError_t launch_step(const DevBatch<float> &b, int waves, int n_sub, int grid, hipStream_t s);
hipError_t launch_advance(int64_t *step, int64_t n, hipStream_t s);
hipError_t launch_energy(const DevBatch<double> &b, double *out, hipStream_t s);
// map (device [n_map]) or NULL: output row i is rod map[i]
hipError_t launch_energy(const DevBatch<float> &b, double *out, hipStream_t s, const int32_t *map = nullptr,
                         int n_map = 0);
// Largest number of co-resident workgroups of the step kernel (occupancy x CUs).
int step_resident_groups(int precision_f32, int waves);
// LDS bytes per workgroup of the step kernel: static, plus the dynamic table of
// the node-interaction kinds (2: connections, 3: walls or contact with
// connections, 4: walls or contact without) with conn_nodes
// connected nodes per tile.
size_t step_lds_bytes(int precision_f32, int waves, int kind, int conn_nodes);

// rod_energy_noalloc's statically allocated device buffer (noalloc.hip): room
// for the energies of NOALLOC_MAX_RODS rods and one int32 result.
constexpr int64_t NOALLOC_MAX_RODS = 262144;
// The buffer's device address on the current device (looked up once per
// device): the energies [5 * NOALLOC_MAX_RODS] and the int32 after them.
int noalloc_scratch(double **energies, int32_t **first_flagged);
// out[0] = smallest r < n with flags[r] != 0, or n (one small kernel).
hipError_t launch_first_flagged(const int32_t *flags, int n, int32_t *out, hipStream_t s);

// Read access to a batch for the surrogate runtime (rod_lib.cpp).
struct BatchView {
    int precision;
    int waves;
    bool extended;             // the batch carries a magnetic couple, gravity or muscle torques
    int32_t n_rods;
    int64_t n_elems, n_slots;
    const int32_t *n;          // host [R]
    const int32_t *rod_slot;   // host [R]
    const double *youngs, *shear_modulus, *density, *radius, *shear_coeff;   // host [R]
    const double *couple_amp, *couple_freq, *couple_phase;                    // host [R][3], [R], [R]
    const int32_t *bc_start, *bc_end;                                         // host [R]
    double dt, time;           // step and current time
    DevBatch<float> f32;       // device pointers (FP32 batches)
    size_t state_bytes, tail_bytes;
};
int batch_view(const rod_batch_opaque *b, BatchView *v);
// Advance the batch's clock by n steps without stepping (the learned coarse step).
int batch_advance_clock(rod_batch_opaque *b, int64_t n, hipStream_t s);
// n plain steps of the rods with active[r] != 0 (device [R]), direct launches
// over the n_list tiles of tile_list (device) that hold those rods.
int batch_step_masked(rod_batch_opaque *b, int64_t n, const int32_t *active, const int32_t *tile_list, int n_list,
                      hipStream_t s);
// Set the batch's clock to time t with its step counter at 0 (direct launches afterwards).
int batch_set_time(rod_batch_opaque *b, double t, hipStream_t s);
hipError_t launch_set_step(int64_t *step, int64_t value, hipStream_t s);

}  // namespace rodk
