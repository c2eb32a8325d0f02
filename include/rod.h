/*
 * rod.h -- C boundary of the MI355X (gfx950) discrete Cosserat-rod library.
 *
 * The library advances many independent elastic rods with the explicit
 * position-Verlet step of the discrete Cosserat model (Elastica++, Methods,
 * "Cosserat rod dynamics", Eq. 1a and 1b; time stepping as the multi-stage
 * symplectic Verlet scheme of Results, "Performance-oriented software
 * design").  Every step of the path runs in HIP kernels on the GPU; the host
 * side only validates, packs and schedules.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: ROD_OK (0) or a negative ROD_E* code.  No C++ exception
 *    crosses this boundary.  rod_last_error() returns a thread-local message
 *    for the last non-zero return (and for warnings attached to ROD_OK).
 *  - Layout of rod data (all FP64, C order):
 *      rod r has n_r elements, n_r + 1 nodes and n_r - 1 Voronoi points;
 *      node j of rod r is row  (sum_{q<r} (n_q + 1)) + j  of a node array,
 *      element i is row         (sum_{q<r} n_q) + i       of an element array,
 *      Voronoi point k is row   (sum_{q<r} (n_q - 1)) + k of a Voronoi array.
 *      position, velocity: [N_nodes][3] lab frame (m, m/s)
 *      director:           [N_elems][3][3], row a = director d_{a+1} in lab
 *                          coordinates (the row matrix Q = {d1,d2,d3}^T)
 *      omega:              [N_elems][3] angular velocity in the material
 *                          frame, omega = ax(Q dQ^T/dt)
 *  - Ownership: rod_batch_create copies everything it needs into device
 *    memory it owns; the caller keeps its arrays.  Output buffers belong to
 *    the caller.  A handle is valid until rod_batch_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  rod_step only enqueues work; rod_energy, rod_get_state,
 *    rod_set_state and rod_get_flags synchronise the stream.
 *  - Precision: inputs are always FP64.  ROD_F32 batches round them once at
 *    creation (round to nearest even) and store, per element, the edge
 *    vector r_{i+1} - r_i and, per rod, the first node relative to an FP64
 *    origin (that node at creation); rod_get_state sums the edges in FP64.
 *  - Not thread-safe per handle: calls on one handle must not overlap.
 */
#ifndef ROD_H
#define ROD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ROD_OK = 0,
    ROD_EINVAL = -1,        /* invalid argument (see rod_last_error) */
    ROD_ENOMEM = -2,        /* device or host allocation failed */
    ROD_EDEVICE = -3,       /* a HIP runtime call failed */
    ROD_ENONFINITE = -4,    /* a rod's state became NaN/Inf (see rod_get_flags) */
    ROD_EUNSUPPORTED = -5   /* valid but outside what the library supports */
};

enum { ROD_F64 = 0, ROD_F32 = 1 };
enum { ROD_FREE = 0, ROD_CLAMPED = 1 };

/* Longest rod (elements) one workgroup tile can hold. */
#define ROD_MAX_ELEMS 512
#define ROD_MAX_WALLS 8

typedef struct rod_batch rod_batch;

/*
 * Problem description (Methods, "Cosserat rod dynamics": centreline r,
 * directors Q, angular velocity omega, density rho, Young's and shear moduli
 * E and G, shear coefficient alpha_c, cross-section; external force f and
 * couple c; boundary conditions per property (4) of that section).
 * The cross-section is a solid circle of the given radius:
 *   A = pi r^2, I1 = I2 = pi r^4 / 4, I3 = I1 + I2,
 *   S = diag(alpha_c G A, alpha_c G A, E A), B = diag(E I1, E I2, G I3).
 */
typedef struct {
    int32_t n_rods;                  /* R >= 1 */
    const int32_t *n_elems;          /* [R], each in [1, ROD_MAX_ELEMS] */
    const double *position;          /* [N_nodes][3] required */
    const double *velocity;          /* [N_nodes][3] required */
    const double *director;          /* [N_elems][3][3] required, in SO(3) within 1e-8 */
    const double *omega;             /* [N_elems][3] required */
    const double *rest_length;       /* [N_elems] > 0, or NULL: chord lengths of `position` */
    const double *rest_kappa;        /* [N_vor][3] rest curvature, or NULL: 0 */
    const double *density;           /* [R] rho > 0 (kg/m^3) */
    const double *youngs;            /* [R] E > 0 (Pa) */
    const double *shear_modulus;     /* [R] G > 0 (Pa) */
    const double *radius;            /* [R] > 0 (m) */
    const double *shear_coeff;       /* [R] alpha_c > 0 */
    const double *damping;           /* [R] gamma >= 0 (1/s): a -= gamma v, alpha -= gamma omega; or NULL: 0 */
    const int32_t *bc_start;         /* [R] ROD_FREE / ROD_CLAMPED at s = 0, or NULL: free */
    const int32_t *bc_end;           /* [R] ROD_FREE / ROD_CLAMPED at s = L, or NULL: free */
    const double *end_force;         /* [R][3] constant lab-frame force on the last node (N), or NULL */
    const double *couple_amp;        /* [R][3] distributed couple amplitude per unit length,
                                        material frame (N m/m), or NULL */
    const double *couple_freq;       /* [R] Hz (with couple_amp): c(t) = amp sin(2 pi f t + phase) */
    const double *couple_phase;      /* [R] rad (with couple_amp) */
    double dt;                       /* time step h > 0 (s) */
    double t0;                       /* time of the initial state (s) */
    int32_t precision;               /* ROD_F64 or ROD_F32 */
    int32_t substeps;                /* steps per kernel launch; 0: all steps of a rod_step call
                                        (autotune: 0 = tuned) */
    int32_t tile_waves;              /* wave64s per workgroup tile (1, 2, 4, 8); 0: smallest that fits
                                        (autotune: 0 = tuned) */
    int32_t inputs_on_device;        /* 1: every pointer above is device memory; 0: host */
    int32_t autotune;                /* 1: choose every tile parameter given as 0 by timing (below) */
    /* Magnetic couple (Methods, "Magnetized filaments", Eq. 2): element i of
     * the batch carries a magnetization m_i per unit length in its material
     * frame, and every rod sits in one homogeneous lab-frame field
     *   b(t) = field[0:3] + field[3:6] cos(2 pi field_freq t) + field[6:9] sin(2 pi field_freq t)  (T),
     * evaluated at the time of each kick; the couple per unit length
     * m_i x (Q_i b(t)) joins c.  NULL magnetization: no magnetic couple (the
     * step then runs the kernel without the term, and field is ignored). */
    const double *magnetization;     /* [N_elems][3] (A m), or NULL */
    double field[9];                 /* b0, bc, bs (lab frame) */
    double field_freq;               /* Hz */
    /* Gravity (Results, "Active matter": the rods
     * settle under gravity): a uniform lab-frame acceleration g adds m_j g to
     * the force on every node (Eq. 1a's f); its work joins W_ext. */
    double gravity[3];               /* g (m/s^2); zero: none */
    /* Muscle torques (same section: internal, net-zero torques prescribed as a
     * travelling wave after the snake-locomotion model it cites).  An active
     * moment at Voronoi point k of rod r,
     *   m_k(t) = beta_k sin(2 pi f_r t - q_r s_k + phi_r) axis_r   (material frame),
     * with s_k the rest arc length from the rod's first node to the Voronoi
     * point, adds to the internal moment B kappa / e^3 of Eq. 1b (so it enters
     * both d/ds(.) and kappa x (.), and sums to zero over a rod).  Evaluated
     * at the time of each kick. */
    const double *muscle_amp;        /* [N_vor] beta_k (N m), or NULL: no muscle torque */
    const double *muscle_axis;       /* [R][3] material-frame axis (with muscle_amp; its length scales beta) */
    const double *muscle_freq;       /* [R] f = 1 / period (Hz) */
    const double *muscle_wavenumber; /* [R] q = 2 pi / wavelength (rad/m) */
    const double *muscle_phase;      /* [R] phi (rad) */
    /* Rod-rod connections (Results, "Magnetized filament assemblies": components
     * joined point-wise, backbones by distributed lateral connections).  Each
     * connection is a central spring-dashpot between node conn_node[c][0] of rod
     * conn_rod[c][0] and node conn_node[c][1] of rod conn_rod[c][1] (node indices
     * 0..n of their rods): with l the distance between the two nodes and e the
     * unit vector from the first to the second, the first node receives
     *   [k (l - l0) + c dl/dt] e   (pre-kick velocities, at the kick time)
     * and the second the opposite; half of its potential 1/2 k (l - l0)^2 joins
     * each rod's W_ext.  Rods joined directly or through other rods are packed
     * into one workgroup tile, so a connected group must fit a tile (at most
     * 512 elements; ROD_EUNSUPPORTED otherwise, or when tile_waves is too small
     * for it). */
    int32_t n_connections;           /* C >= 0 */
    const int32_t *conn_rod;         /* [C][2] rod indices */
    const int32_t *conn_node;        /* [C][2] node indices within the rods */
    const double *conn_k;            /* [C] spring stiffness >= 0 (N/m) */
    const double *conn_c;            /* [C] dashpot coefficient >= 0 (N s/m) */
    const double *conn_rest;         /* [C] rest distance >= 0 (m) */
    /* Planar walls (Results, "Active matter" and "Fibrous granular materials":
     * filaments confined by boundaries and in frictional contact with them).
     * Wall w is the solid half-space n.x < d (walls[w] = {nx, ny, nz, d}, n a
     * unit normal); every node is a sphere of its rod's radius.  While a node
     * penetrates a wall by delta = radius - (n.x - d) > 0 it receives the
     * normal force f_n n, f_n = delta (wall_k - wall_c (n.v)) (damping grows
     * with the penetration, so the force is continuous at contact onset),
     * when f_n > 0, and
     * the friction -wall_mu f_n v_t / max(|v_t|, wall_vslip) against its
     * tangential velocity v_t (Coulomb, viscous below the slip speed), with
     * pre-kick velocities at the kick time.  The penalty potential
     * 1/2 wall_k delta^2 joins W_ext.  Below the slip speed the friction is a
     * damper of coefficient wall_mu f_n / wall_vslip: the explicit step needs
     * wall_mu f_n h / (m wall_vslip) well below 2 for node masses m (the
     * contact frequency sqrt(wall_k / m) enters the stability warning).
     * The same law, with the same four parameters, acts between the nodes of
     * different rods when rod_contact is set (below). */
    int32_t n_walls;                 /* 0..ROD_MAX_WALLS */
    const double *walls;             /* [n_walls][4], host memory always */
    double wall_k;                   /* N/m >= 0 */
    double wall_c;                   /* N s/m^2 >= 0 */
    double wall_mu;                  /* >= 0 */
    double wall_vslip;               /* m/s > 0 (with walls or rod contact) */
    /* Rod-rod contact (Results, "Fibrous granular materials"; the collision
     * engine the paper names as future work).  With rod_contact = 1 every
     * node is a sphere of its rod's radius, and two nodes of different rods
     * whose centres are closer than the sum of their radii each receive the
     * wall law above with the overlap delta = r_a + r_b - |x_a - x_b|, the
     * normal (x_a - x_b)/|x_a - x_b| and the relative velocity v_a - v_b (so
     * the pair's forces are equal and opposite); half of each pair's penalty
     * potential 1/2 wall_k delta^2 joins each rod's W_ext.  A rod does not
     * touch itself.  Pairs are found by a hashed uniform grid over the node
     * positions (cells of twice the largest radius), every step or, with
     * Verlet lists (contact_skin, below), when the lists need a rebuild.
     * With rod_contact = 2 every element is a capsule, the segment between
     * its two nodes dilated by its rod's radius: the same law acts between the
     * closest points of two elements' segments (the point velocities
     * interpolated along each element), and the force on an element goes to
     * its nodes in the shares (1 - s) and s of the closest point's parameter s
     * along it.  Each pair is evaluated once, in (rod, element) order, and the
     * other element takes the exact negative, so the pair's forces cancel
     * bit for bit.  Elements of one rod touch when the rest lengths of the
     * elements between them add up to at least the diameter (self-contact of
     * a folded rod).  The grid bins element midpoints in cells of 1.25 times
     * the longest rest length plus twice the largest radius: contacts of
     * elements stretched by more than a quarter of their rest length can be
     * missed, and such a rod is flagged (ROD_FLAG_STRETCHED, rod_get_flags).
     * Both modes: each step is one launch sequence, so substeps must be 0 or
     * 1 (one step per launch); FP32 batches sum their node positions along
     * each rod in FP64 for the grid; each grid cell's entries are sorted by
     * node (element) before the forces are summed, so runs are bitwise
     * repeatable and independent of tile_waves. */
    int32_t rod_contact;             /* 0, 1 (node spheres) or 2 (element capsules) */
    /* Verlet lists.  With a skin s > 0 the grid (cells grown by s) lists,
     * for every node (rod_contact = 1), the nodes of other rods closer than
     * its radius plus the largest radius plus s, or, for every element
     * (rod_contact = 2), the elements it may touch whose segments are closer
     * than the two radii plus s; the grid pass then runs again only in a
     * step where some node has moved more than s/2 since (the distance
     * between two nodes or two segments changes by at most the sum of their
     * moves), or where a list would have held more than 32 partners (that
     * item's contacts are summed in grid order and the next step builds
     * again).  Every step sums each item's contacts over its list in
     * increasing node (element slot) order, so the results do not depend on
     * s or on when the lists were built (bit for bit, while no list
     * overflows).  0: s = a fifth of the largest radius; < 0: no lists (the
     * grid pass every step, contacts summed in grid order).  Not finite:
     * ROD_EINVAL. */
    double contact_skin;             /* m */
} rod_batch_desc;

/* One timed candidate of the autotuner. */
typedef struct {
    int32_t tile_waves;
    int32_t substeps;
    double ns_per_element_step;      /* device time per element-step of the trial */
} rod_tune_trial;

#define ROD_MAX_TUNE_TRIALS 12

/*
 * Create a batch: validate, derive the per-element constants in FP64, pack
 * the rods into workgroup tiles (whole rods per tile, best-fit decreasing),
 * and upload.  Errors: ROD_EINVAL (n_elems outside [1, ROD_MAX_ELEMS], a
 * NULL required array, dt <= 0, rho/E/G/radius/alpha_c <= 0, damping < 0,
 * a director farther than 1e-8 from SO(3) or with det < 0, a zero-length
 * element or rest length <= 0, couple_amp without freq/phase, muscle_amp
 * without axis/freq/wavenumber/phase, a magnetization, field, field_freq,
 * gravity or muscle input that is not finite, a connection naming a rod or
 * node outside the batch, joining a node to itself, or with k, c or l0
 * negative or not finite; n_walls outside [0, ROD_MAX_WALLS], a wall normal
 * not of unit length within 1e-9, wall_k, wall_c or wall_mu negative,
 * wall_vslip <= 0, rod_contact not 0, 1 or 2, rod_contact with substeps > 1,
 * contact_skin not finite),
 * ROD_ENOMEM, ROD_EDEVICE, ROD_EUNSUPPORTED (tile_waves too small for the
 * longest rod or connected group).
 * A time step above the explicit stability estimate is reported through
 * rod_last_error with ROD_OK.
 */
int rod_batch_create(const rod_batch_desc *desc, void *stream, rod_batch **out);

/*
 * The autotuner (desc->autotune = 1).  Candidates: tile_waves in {1, 2, 4, 8}
 * that hold the longest rod (when tile_waves = 0) times substeps in
 * {50, 200, 1000} (when substeps = 0; {1} with rod contact).  Each tile width is packed into a
 * scratch batch of the same rods; each candidate runs one warm-up launch and
 * then 1000 timed steps (HIP events on a private stream; the scratch state is
 * discarded), and the fastest per element-step is kept.  Tile width does not
 * change results; substeps per launch change them at round-off (the half
 * drifts of consecutive steps are fused inside a launch).  rod_batch_tuning
 * returns the trials (n_trials = 0 without autotuning).
 */
int rod_batch_tuning(const rod_batch *b, rod_tune_trial *trials, int32_t max_trials, int32_t *n_trials);

/*
 * Advance every rod by n_steps >= 0 position-Verlet steps of size dt
 * (Results, "Performance-oriented software design"): per step a half drift
 * r += h/2 v, Q <- exp(-h/2 [omega]x) Q; the kick v += h a, omega += h alpha
 * with a, alpha from Eq. 1a / 1b at time t_n + h/2; a second half drift; the
 * clamped ends' kinematic constraints after every stage.  The steps run as
 * ceil(n_steps / substeps) launches of one persistent kernel whose tiles
 * keep the rods' state on chip across the substeps; the launch sequence is
 * captured once per distinct n_steps into a HIP graph and replayed.
 * Asynchronous on `stream`.  ROD_EINVAL for n_steps < 0 or a NULL handle.
 */
int rod_step(rod_batch *b, int64_t n_steps, void *stream);

/*
 * Per-rod energies, out[R][5] (host, FP64), synchronising `stream`:
 *   T_lin   = 1/2 sum_j m_j |v_j|^2
 *   T_rot   = 1/2 sum_i omega_i . J_i omega_i / e_i   (Eq. 1b's rho I omega / e)
 *   U_shear = 1/2 sum_i sigma_i . S sigma_i lh_i
 *   U_bend  = 1/2 sum_k (kappa_k - kappa0_k) . B_k (kappa_k - kappa0_k) Dh_k
 *   W_ext   = -sum f . (r_last - r_last(0)) - sum_j m_j g . (r_j - r_j(0))
 *             + half of 1/2 k (l - l0)^2 of every connection at the rod
 *             + 1/2 wall_k delta^2 of every node in contact with a wall
 *             + half of 1/2 wall_k delta^2 of every node pair in rod contact
 *                      (the end force, gravity, connections, walls, contacts)
 * The distributed, magnetic and muscle couples have no energy column.  Returns ROD_ENONFINITE if any rod is flagged non-finite.
 */
int rod_energy(rod_batch *b, double *out, void *stream);

/*
 * rod_energy for callers that cannot allocate device memory (code that must
 * not call hipMalloc: serving loops, harnesses that forbid allocation).  Same
 * arguments, result and errors as rod_energy, bit for bit; the per-rod
 * energies are staged in a statically allocated device buffer of the library
 * instead of one allocated with the batch.  No device memory is allocated or
 * freed (the buffer's address is looked up once per device, on the first call
 * there).
 * Limit: batches of at most 262,144 rods (the buffer holds 5 doubles per rod,
 * 10 MiB, and stays allocated on every device the library runs on until the
 * process ends); larger batches get ROD_EINVAL.  Call with the batch's device
 * current.  All calls on one device share the buffer: calls that overlap in
 * time on one device (other host threads, other streams) race and must not
 * be made.
 */
int rod_energy_noalloc(rod_batch *b, double *out, void *stream);

/* Copy the state back into caller-owned host arrays in the layout above (any
 * pointer may be NULL to skip it); *t receives the current time.
 * Synchronises `stream`.  ROD_ENONFINITE if any rod is flagged. */
int rod_get_state(rod_batch *b, double *position, double *velocity, double *director,
                  double *omega, double *t, void *stream);

/* Overwrite the state (host arrays, layout above; NULL keeps a field) and the
 * time.  Constraints of clamped ends are re-imposed (their node and element
 * keep the values captured at creation, with zero velocities).
 * Synchronises `stream`.  Clears the non-finite flags. */
int rod_set_state(rod_batch *b, const double *position, const double *velocity,
                  const double *director, const double *omega, double t, void *stream);

/* Per-rod flags (host int32 [R], bits): ROD_FLAG_NONFINITE = NaN/Inf seen at
 * the end of a launch (the synchronising calls then return ROD_ENONFINITE; a
 * non-finite rod can make the next rods of its workgroup tile non-finite in
 * later steps, and flagged, since a rod's first Voronoi point takes the
 * previous rod's values times zero stiffness; contact carries no NaN);
 * ROD_FLAG_STRETCHED = with capsule contact (rod_contact = 2), an element of
 * the rod was longer than 1.25 times the longest rest length when the contact
 * grid binned it, so contacts of that element may have been missed (the state
 * stays valid; no call fails for it).  Synchronises `stream`.  rod_set_state
 * clears both. */
enum { ROD_FLAG_NONFINITE = 1, ROD_FLAG_STRETCHED = 2 };
int rod_get_flags(rod_batch *b, int32_t *nonfinite, void *stream);

/* Sizes and the chosen launch shape: info[0] rods, [1] elements, [2] tiles,
 * [3] tile_waves, [4] substeps per launch (0 = whole call), [5] precision,
 * [6] slots (tiles * 64 * tile_waves), [7] steps taken so far. */
int rod_batch_info(const rod_batch *b, int64_t *info);

/* Verlet-list counters of a batch with rod contact and a skin > 0 (all
 * zero otherwise): out[0] contact passes (one per step, one per energy call),
 * [1] passes that rebuilt the lists, [2] builds at which a list overflowed
 * (its item's contacts were summed in grid order, and the next pass built
 * again), [3] the most partners one node or element had at a build, [4] the
 * list capacity (32).  Counters wrap at 2^32.  Synchronises `stream`. */
int rod_contact_stats(rod_batch *b, int64_t *out, void *stream);

void rod_batch_destroy(rod_batch *b);

/* Thread-local message for the last non-zero return or warning ("" if none). */
const char *rod_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ROD_H */
