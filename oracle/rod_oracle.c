/*
 * rod_oracle.c -- plain FP64 CPU oracle of the discrete Cosserat-rod step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: every derived quantity is
 * recomputed here from the raw material parameters, one rod at a time, in the
 * most direct form, with the C library's sqrt/sin/cos/atan2.
 *
 * Model (Elastica++, Methods, "Cosserat rod dynamics"):
 *   centreline r(s,t), row director matrix Q = {d1,d2,d3}^T, local vectors
 *   vbar = Q v; strains sigma = Q(r' - d3), kappa = ax(Q dQ^T/ds),
 *   omega = ax(Q dQ^T/dt); e = |r'|; B = diag(EI1, EI2, G(I1+I2)),
 *   S = diag(alpha_c G A, alpha_c G A, E A), I = diag(I1, I2, I1+I2);
 *   linear momentum  (Eq. 1a): rho A r_tt = d/ds(Q^T S sigma / e) + f
 *   angular momentum (Eq. 1b): (rho I / e) omega_t = d/ds(B kappa / e^3)
 *        + kappa x B kappa / e^3 + Q t x S sigma + (rho I omega / e) x omega
 *        + (rho I omega / e^2) e_t + c.
 * The paper defers its discretisation to a supplement that is not available;
 * the discretisation below is the staggered one of the cited discrete model
 * (nodes carry r, v; elements carry Q, omega; Voronoi points between adjacent
 * elements carry kappa), with these readings:
 *   - element i joins nodes i and i+1; rest length lh_i; Voronoi k joins
 *     elements k and k+1 with rest length Dh_k = (lh_k + lh_{k+1})/2;
 *   - sigma_i = Q_i (r_{i+1}-r_i)/lh_i - e3   (Q d3 = e3 for orthonormal Q);
 *   - kappa_k = log(Q_k Q_{k+1}^T) / Dh_k, the rotation vector of the relative
 *     rotation evaluated with atan2;
 *   - difference operator: node j receives n_j - n_{j-1} (zero outside);
 *     element i receives M_i - M_{i-1}; averaging operator: element i
 *     receives (y_{i-1} + y_i)/2 (zero outside);
 *   - solid circular section: A = pi r^2, I1 = I2 = pi r^4 / 4;
 *   - lumped masses m_j = (rho A lh_{j-1} + rho A lh_j)/2;
 *     element inertia J_i = rho I lh_i;
 *   - Voronoi bending stiffness = rest-length weighted mean of the two
 *     elements' B;
 *   - rest strains: sigma0 = 0, kappa0 given or 0;
 *   - linear damping: a -= gamma v, alpha -= gamma omega;
 *   - velocity-dependent terms use the pre-kick velocities;
 *   - time integration: position Verlet (Results, "Performance-oriented
 *     software design": a multi-stage symplectic Verlet scheme whose every
 *     stage re-imposes the kinematic constraints):
 *       half drift (r += h/2 v, Q <- exp(-h/2 [omega]x) Q), constraints,
 *       kick (v += h a, omega += h alpha) at t_n + h/2, constraints,
 *       half drift, constraints;
 *   - clamped end: node position and element director reset to their initial
 *     values, node velocity and element angular velocity set to zero;
 *   - magnetic couple (Methods, "Magnetized filaments", Eq. 2): element i
 *     carries a magnetization m_i per unit length in its material frame; a
 *     homogeneous lab field b(t) = b0 + bc cos(2 pi f t) + bs sin(2 pi f t),
 *     evaluated at the kick time, adds m_i x (Q_i b) to the couple c;
 *   - gravity (Results, "Active matter"): nodal force m_j g;
 *   - muscle torques (same section; a travelling wave of internal, net-zero
 *     torques): an active moment beta_k sin(2 pi f t - q s_k + phi) axis at
 *     Voronoi point k, s_k its rest arc length from the first node, added to
 *     the internal moment B kappa / e^3 (so it enters both the difference
 *     and the kappa x M terms), evaluated at the kick time;
 *   - connections (Results, "Magnetized filament assemblies": components joined
 *     point-wise and by distributed lateral connections): a central
 *     spring-dashpot between two nodes, force on the first
 *     [k (l - l0) + c dl/dt] (x_b - x_a)/l, the opposite on the second,
 *     with pre-kick velocities (nothing while the two nodes coincide); its
 *     potential 1/2 k (l - l0)^2 is split evenly between the two rods' W_ext.
 *   - planar walls (Results, "Active matter" and "Fibrous granular materials":
 *     filaments confined by and in frictional contact with boundaries; the
 *     contact model itself is in the supplement, which is not available): each
 *     node is a sphere of the rod's radius; penalty normal force
 *     delta (k - c v_n) while it penetrates a wall by delta and that force is
 *     positive (damping grows with the penetration, so the force is continuous
 *     at contact onset), Coulomb friction mu f_n against the tangential velocity,
 *     regularised as viscous below a slip speed; the penalty potential
 *     1/2 k delta^2 joins W_ext.
 *   - rod-rod contact (Results, "Fibrous granular materials" and the
 *     collision engine the paper names as future work; the contact law is in
 *     the unavailable supplement): nodes are spheres of their rod's radius,
 *     as for the walls; two nodes of different rods touch when their centres
 *     are closer than the sum of the radii, and each feels the wall law with
 *     the overlap of the two spheres, the normal from the other's centre and
 *     their relative velocity (so the pair's forces are equal and opposite);
 *     half of each pair's penalty potential goes to each rod's W_ext.  A rod
 *     does not touch itself.  (Crossing rods whose elements are longer than
 *     their diameters can pass between nodes.)
 *   - segment contact (rod_contact = 2; the same sources): every element is a
 *     capsule, the segment between its two nodes dilated by the rod's radius.
 *     Two capsules touch when the distance between the closest points P (on
 *     element a, parameter s) and Q (on element b, parameter t) of their
 *     segments is below the sum of the radii; element a then feels the wall
 *     law with that overlap, the normal from Q to P and the relative velocity
 *     of the two points (node velocities interpolated with the same
 *     parameters), and the force is shared by its two nodes as (1 - s) and s
 *     (so its moment about any point is that of the force at P).  Elements of
 *     different rods touch, and so do elements of one rod when the rest lengths
 *     of the elements between them add up to at least the rod's diameter (in
 *     the straight rest state such capsules do not overlap; closer ones always
 *     would).  Half of each pair's penalty potential goes to each rod.
 * Rods joined by connections or in contact are advanced together (one batch
 * step), the coupling forces from the state of all rods at the kick time.
 *
 * FP32 mirror.  The same source compiled with -DORC_F32 (and
 * -fsingle-precision-constant, so that literals do not lift expressions to
 * FP64) carries out every operation of the rod step above in IEEE single
 * precision: the reference for what FP32 arithmetic of this method gives,
 * against which an FP32 implementation's discrepancy from the FP64 oracle is
 * judged.  Its inputs (material constants, rest lengths and curvatures, loads,
 * magnetization, muscle amplitudes, initial directors) are FP32 arrays, i.e.
 * rounded once from FP64.  What stays FP64 in the mirror:
 *   - time and the phases of the time-dependent loads (sin(2 pi f t + phi)
 *     evaluated in FP64, then rounded);
 *   - positions: a rod's nodes are held as an FP64 origin (its first node at
 *     creation) plus, in FP32, the first node relative to it (the anchor) and
 *     the element edge vectors r_{i+1} - r_i.  The half drift
 *     r_j += h/2 v_j becomes anchor += h/2 v_0, edge_i += h/2 (v_{i+1} - v_i),
 *     the same update in exact arithmetic; FP32 absolute positions would
 *     round every drift increment against the rod's whole extent, which is
 *     not a property of the method;
 *   - the node-interaction laws (walls, connections, rod-rod contact), which
 *     are evaluated in FP64 on node positions summed from the FP32 state,
 *     their forces rounded to FP32.
 * In the FP32 build the position array of a rod holds the anchor in row 0 and
 * edge i in row i + 1, and a clamped far end is imposed by setting the last
 * edge so that node n sits at its initial position.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_F32
typedef float real;
#define SQRT sqrtf
#define SIN sinf
#define COS cosf
#define ATAN2 atan2f
#define POW powf
#else
typedef double real;
#define SQRT sqrt
#define SIN sin
#define COS cos
#define ATAN2 atan2
#define POW pow
#endif
/* 2 pi in FP64 in both builds (a literal would be single precision in the
 * FP32 build) */
#define ORC_TWO_PI (8.0 * atan(1.0))

typedef struct {
    int32_t n_rods;
    const int32_t *n_elems;          /* [R] */
    const real *density;             /* [R] rho */
    const real *youngs;              /* [R] E */
    const real *shear_modulus;       /* [R] G */
    const real *radius;              /* [R] */
    const real *shear_coeff;         /* [R] alpha_c */
    const real *damping;             /* [R] gamma, 1/s */
    const int32_t *bc_start;         /* [R] 1: clamped at s = 0 */
    const int32_t *bc_end;           /* [R] 1: clamped at s = L */
    const real *rest_length;         /* [N_e] */
    const real *rest_kappa;          /* [N_v][3] or NULL */
    const real *node_force;          /* [N_n][3] or NULL: constant external nodal force */
    const real *couple_amp;          /* [N_e][3] or NULL: couple per unit length, material frame */
    const double *couple_freq;       /* [R] Hz (used with couple_amp) */
    const double *couple_phase;      /* [R] rad */
    const double *pos0;              /* [N_n][3] initial positions (constraints, work of f) */
    const real *dir0;                /* [N_e][9] initial directors (constraints) */
    double dt;
    double t0;                       /* time at step 0 */
    int32_t drop_term;               /* 0 in normal use; k > 0 removes term k (mutation tests) */
    const real *magnetization;       /* [N_e][3] or NULL: magnetization per unit length, material frame */
    double field[9];                 /* b(t) = field[0:3] + field[3:6] cos(2 pi f t) + field[6:9] sin(2 pi f t) */
    double field_freq;               /* f, Hz */
    double gravity[3];               /* g, m/s^2: nodal force m_j g */
    const real *muscle_amp;          /* [N_v] or NULL: active moment amplitude beta_k */
    const real *muscle_axis;         /* [R][3] material-frame axis */
    const double *muscle_freq;       /* [R] Hz */
    const double *muscle_wavenumber; /* [R] rad/m */
    const double *muscle_phase;      /* [R] rad */
    int32_t n_conn;                  /* node-pair connections */
    const int32_t *conn_node;        /* [C][2] global node indices (rows of the node arrays) */
    const double *conn_k;            /* [C] spring stiffness (N/m) */
    const double *conn_c;            /* [C] dashpot coefficient (N s/m) */
    const double *conn_rest;         /* [C] rest distance (m) */
    int32_t n_walls;                 /* planar boundaries */
    const double *wall;              /* [n_walls][4]: unit normal nx ny nz, offset d (the wall is n.x = d) */
    double wall_k, wall_c, wall_mu, wall_vslip;   /* contact stiffness, damping, friction, slip speed */
    int32_t rod_contact;             /* 1: contact between nodes of different rods (same law); 2: capsule
                                        contact between elements, of different rods and of one rod */
    const double *origin;            /* FP32 build: [R][3] rod origins (first node at creation); else unused */
} orc_rods;

/* ---------------------------------------------------------------- vectors */

static void cross3(const real *a, const real *b, real *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static real dot3(const real *a, const real *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* FP64 dot product (node-interaction laws) */
static double dot3d(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* y = Q x, Q row-major 3x3 */
static void matvec(const real *Q, const real *x, real *y)
{
    for (int a = 0; a < 3; ++a)
        y[a] = Q[3 * a + 0] * x[0] + Q[3 * a + 1] * x[1] + Q[3 * a + 2] * x[2];
}

/* y = Q^T x */
static void matTvec(const real *Q, const real *x, real *y)
{
    for (int b = 0; b < 3; ++b)
        y[b] = Q[0 + b] * x[0] + Q[3 + b] * x[1] + Q[6 + b] * x[2];
}

/* C = A B^T */
static void mat_abt(const real *A, const real *B, real *C)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            C[3 * a + b] = A[3 * a + 0] * B[3 * b + 0] + A[3 * a + 1] * B[3 * b + 1]
                         + A[3 * a + 2] * B[3 * b + 2];
}

/* C = A B */
static void mat_ab(const real *A, const real *B, real *C)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            C[3 * a + b] = A[3 * a + 0] * B[0 + b] + A[3 * a + 1] * B[3 + b]
                         + A[3 * a + 2] * B[6 + b];
}

/* Rotation exp([u]x) by the Rodrigues formula:
 * I + sin(th) [k]x + (1 - cos(th)) [k]x^2 with th = |u|, k = u/th; exp(0) = I. */
static void rodrigues(const real *u, real *E)
{
    real th = SQRT(dot3(u, u));
    for (int i = 0; i < 9; ++i) E[i] = 0.0;
    E[0] = E[4] = E[8] = 1.0;
    if (th == 0.0) return;
    real k[3] = {u[0] / th, u[1] / th, u[2] / th};
    real K[9] = {0.0, -k[2], k[1],
                 k[2], 0.0, -k[0],
                 -k[1], k[0], 0.0};
    real K2[9];
    mat_ab(K, K, K2);
    real s = SIN(th), c1 = 1.0 - COS(th);
    for (int i = 0; i < 9; ++i) E[i] += s * K[i] + c1 * K2[i];
}

/* Rotation vector u with exp([u]x) = R for a rotation matrix R:
 * w = ax(R) = (R32 - R23, R13 - R31, R21 - R12)/2 = sin(th) k,
 * c = (tr R - 1)/2 = cos(th), th = atan2(|w|, c), u = (th/|w|) w.
 * For |w| -> 0 the ratio th/|w| tends to 1 + |w|^2/6. */
static void logmap(const real *R, real *u)
{
    real w[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
    real sw = SQRT(dot3(w, w));
    real c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    real f;
    if (sw < 1e-7 && c > 0.0)
        f = 1.0 + sw * sw / 6.0;   /* next term 3|w|^4/40 is below FP64 resolution */
    else
        f = ATAN2(sw, c) / sw;     /* a half-turn (w = 0, c = -1) has no unique axis */
    u[0] = f * w[0];
    u[1] = f * w[1];
    u[2] = f * w[2];
}

/* ------------------------------------------------------------ one rod view */

typedef struct {
    int n;                       /* elements */
    real rho, E, G, rad, alpha_c, gamma;
    double freq, phase;
    int clamp0, clamp1;
    const real *lh;              /* [n] rest lengths */
    const real *k0;              /* [n-1][3] or NULL */
    const real *fext;            /* [n+1][3] or NULL */
    const real *camp;            /* [n][3] or NULL */
    const double *r0;            /* [n+1][3] */
    const double *org;           /* FP32 build: [3] the rod's origin */
    const real *Q0;              /* [n][9] */
    const real *mag;             /* [n][3] or NULL */
    const double *field;         /* [9] */
    double field_freq;
    const double *grav;          /* [3] */
    const double *fconn;         /* [n+1][3] or NULL: connection forces at this kick */
    int32_t n_walls;
    const double *wall;
    double wall_k, wall_c, wall_mu, wall_vslip;
    const real *mamp;            /* [n-1] or NULL */
    const real *maxis;           /* [3] */
    double mfreq, mwave, mphase;
    int drop;
} rod_view;

static void rod_view_make(const orc_rods *p, int r, int64_t eo, int64_t no, int64_t vo, rod_view *v)
{
    v->n = p->n_elems[r];
    v->rho = p->density[r];
    v->E = p->youngs[r];
    v->G = p->shear_modulus[r];
    v->rad = p->radius[r];
    v->alpha_c = p->shear_coeff[r];
    v->gamma = p->damping ? p->damping[r] : 0.0;
    v->clamp0 = p->bc_start ? p->bc_start[r] : 0;
    v->clamp1 = p->bc_end ? p->bc_end[r] : 0;
    v->freq = p->couple_freq ? p->couple_freq[r] : 0.0;
    v->phase = p->couple_phase ? p->couple_phase[r] : 0.0;
    v->lh = p->rest_length + eo;
    v->k0 = p->rest_kappa ? p->rest_kappa + 3 * vo : NULL;
    v->fext = p->node_force ? p->node_force + 3 * no : NULL;
    v->camp = p->couple_amp ? p->couple_amp + 3 * eo : NULL;
    v->r0 = p->pos0 + 3 * no;
    v->org = p->origin ? p->origin + 3 * r : NULL;
    v->Q0 = p->dir0 + 9 * eo;
    v->mag = p->magnetization ? p->magnetization + 3 * eo : NULL;
    v->field = p->field;
    v->field_freq = p->field_freq;
    v->grav = p->gravity;
    v->fconn = NULL;
    v->n_walls = p->n_walls;
    v->wall = p->wall;
    v->wall_k = p->wall_k;
    v->wall_c = p->wall_c;
    v->wall_mu = p->wall_mu;
    v->wall_vslip = p->wall_vslip;
    v->mamp = p->muscle_amp ? p->muscle_amp + vo : NULL;
    v->maxis = p->muscle_amp ? p->muscle_axis + 3 * r : NULL;
    v->mfreq = p->muscle_amp ? p->muscle_freq[r] : 0.0;
    v->mwave = p->muscle_amp ? p->muscle_wavenumber[r] : 0.0;
    v->mphase = p->muscle_amp ? p->muscle_phase[r] : 0.0;
    v->drop = p->drop_term;
}

/* Section and constitutive constants of one rod. */
typedef struct {
    real A, I1, I2, I3;          /* area, second moments */
    real S[3];                   /* shear/stretch stiffness diag */
    real B[3];                   /* bend/twist stiffness diag */
} rod_consts;

static void rod_consts_make(const rod_view *v, rod_consts *c)
{
    c->A = M_PI * v->rad * v->rad;
    c->I1 = M_PI * POW(v->rad, 4) / 4.0;
    c->I2 = c->I1;
    c->I3 = c->I1 + c->I2;
    c->S[0] = v->alpha_c * v->G * c->A;
    c->S[1] = v->alpha_c * v->G * c->A;
    c->S[2] = v->E * c->A;
    c->B[0] = v->E * c->I1;
    c->B[1] = v->E * c->I2;
    c->B[2] = v->G * c->I3;
}

/* Workspace for one rod of up to nmax elements. */
typedef struct {
    real *l, *e, *t, *edot, *sig, *Ssig, *nint, *kap, *M, *y, *eps;
} rod_work;

static int work_alloc(rod_work *w, int nmax)
{
    size_t ne = (size_t)nmax;
    w->l = malloc(ne * sizeof(real));
    w->e = malloc(ne * sizeof(real));
    w->t = malloc(3 * ne * sizeof(real));
    w->edot = malloc(ne * sizeof(real));
    w->sig = malloc(3 * ne * sizeof(real));
    w->Ssig = malloc(3 * ne * sizeof(real));
    w->nint = malloc(3 * ne * sizeof(real));
    w->kap = malloc(3 * ne * sizeof(real));
    w->M = malloc(3 * ne * sizeof(real));
    w->y = malloc(3 * ne * sizeof(real));
    w->eps = malloc(ne * sizeof(real));
    return (w->l && w->e && w->t && w->edot && w->sig && w->Ssig && w->nint && w->kap && w->M
            && w->y && w->eps) ? 0 : -1;
}

static void work_free(rod_work *w)
{
    free(w->l); free(w->e); free(w->t); free(w->edot); free(w->sig); free(w->Ssig);
    free(w->nint); free(w->kap); free(w->M); free(w->y); free(w->eps);
}

/* Kinematics and strains of one rod at positions r, velocities v, directors Q:
 * l, e, t, edot per element; sigma, S sigma, internal force n per element;
 * eps, kappa per Voronoi point.  Returns nothing; fills w. */
static void rod_kinematics(const rod_view *rv, const rod_consts *c, const real *r,
                           const real *v, const real *Q, rod_work *w)
{
    const int n = rv->n;
    for (int i = 0; i < n; ++i) {
        real dr[3], dv[3];
        for (int a = 0; a < 3; ++a) {
#ifdef ORC_F32
            dr[a] = r[3 * (i + 1) + a];   /* the edge itself */
#else
            dr[a] = r[3 * (i + 1) + a] - r[3 * i + a];
#endif
            dv[a] = v ? v[3 * (i + 1) + a] - v[3 * i + a] : 0.0;
        }
        real l = SQRT(dot3(dr, dr));
        w->l[i] = l;
        w->e[i] = l / rv->lh[i];
        for (int a = 0; a < 3; ++a) w->t[3 * i + a] = dr[a] / l;
        w->edot[i] = dot3(&w->t[3 * i], dv) / rv->lh[i];
        /* sigma = Q dr / lh - e3 */
        real qdr[3];
        matvec(&Q[9 * i], dr, qdr);
        w->sig[3 * i + 0] = qdr[0] / rv->lh[i];
        w->sig[3 * i + 1] = qdr[1] / rv->lh[i];
        w->sig[3 * i + 2] = qdr[2] / rv->lh[i] - 1.0;
        for (int a = 0; a < 3; ++a) w->Ssig[3 * i + a] = c->S[a] * w->sig[3 * i + a];
        /* n = Q^T S sigma / e (lab frame) */
        real qs[3];
        matTvec(&Q[9 * i], &w->Ssig[3 * i], qs);
        for (int a = 0; a < 3; ++a) w->nint[3 * i + a] = qs[a] / w->e[i];
    }
    for (int k = 0; k + 1 < n; ++k) {
        real Dh = 0.5 * (rv->lh[k] + rv->lh[k + 1]);
        w->eps[k] = 0.5 * (w->l[k] + w->l[k + 1]) / Dh;
        real R[9], u[3];
        mat_abt(&Q[9 * k], &Q[9 * (k + 1)], R);
        logmap(R, u);
        for (int a = 0; a < 3; ++a) w->kap[3 * k + a] = u[a] / Dh;
    }
}

/* Contact of a node (sphere of the rod's radius) with the planar walls: a
 * penalty normal force delta (k - c v_n) along the wall normal (linear spring
 * with damping proportional to the penetration, which keeps the force
 * continuous at contact onset) while the node penetrates by
 * delta = radius - (n.x - d) and the normal force is positive,
 * and Coulomb friction -mu f_n v_t / max(|v_t|, v_slip) against the tangential
 * velocity (viscous below the slip speed).  Adds to f; returns the penalty
 * potential 1/2 k delta^2 of the contacts. */
static double wall_force(const rod_view *rv, const double *x, const double *v, double *f)
{
    double pot = 0.0;
    for (int w = 0; w < rv->n_walls; ++w) {
        const double *nw = &rv->wall[4 * w];
        const double delta = rv->rad - (dot3d(nw, x) - nw[3]);
        if (!(delta > 0.0)) continue;
        pot += 0.5 * rv->wall_k * delta * delta;
        const double vn = dot3d(nw, v);
        const double fn = delta * (rv->wall_k - rv->wall_c * vn);
        if (!(fn > 0.0)) continue;
        double vt[3] = {v[0] - vn * nw[0], v[1] - vn * nw[1], v[2] - vn * nw[2]};
        const double speed = sqrt(dot3d(vt, vt));
        const double g = rv->wall_mu * fn / (speed > rv->wall_vslip ? speed : rv->wall_vslip);
        for (int a = 0; a < 3; ++a) f[a] += fn * nw[a] - g * vt[a];
    }
    return pot;
}

/* Linear accelerations a[n+1][3] and angular accelerations alpha[n][3] of one
 * rod (Eq. 1a and 1b) at state (r, v, Q, om) and time t. */
static void rod_accel(const rod_view *rv, const rod_consts *c, const real *r, const real *v,
                      const real *Q, const real *om, double t, rod_work *w,
                      real *acc, real *alpha)
{
    const int n = rv->n;
    rod_kinematics(rv, c, r, v, Q, w);

    /* bending/twisting moments at Voronoi points */
    for (int k = 0; k + 1 < n; ++k) {
        real Dh = 0.5 * (rv->lh[k] + rv->lh[k + 1]);
        real Bv[3];
        for (int a = 0; a < 3; ++a)
            Bv[a] = (c->B[a] * rv->lh[k] + c->B[a] * rv->lh[k + 1]) / (rv->lh[k] + rv->lh[k + 1]);
        real e3 = w->eps[k] * w->eps[k] * w->eps[k];
        real dk[3];
        for (int a = 0; a < 3; ++a)
            dk[a] = w->kap[3 * k + a] - (rv->k0 ? rv->k0[3 * k + a] : 0.0);
        for (int a = 0; a < 3; ++a) w->M[3 * k + a] = Bv[a] * dk[a] / e3;
        /* active muscle moment at Voronoi k (travelling wave in the rest arc
         * length s_k of the point), part of the internal moment */
        if (rv->mamp) {
            double sk = 0.0;
            for (int i = 0; i <= k; ++i) sk += rv->lh[i];
            const real act = rv->mamp[k] * (real)sin(ORC_TWO_PI * rv->mfreq * t - rv->mwave * sk + rv->mphase);
            for (int a = 0; a < 3; ++a) w->M[3 * k + a] += act * rv->maxis[a];
        }
        real kxM[3];
        cross3(&w->kap[3 * k], &w->M[3 * k], kxM);
        for (int a = 0; a < 3; ++a) w->y[3 * k + a] = kxM[a] * Dh;
    }

    /* nodes: Eq. 1a with the difference operator */
#ifdef ORC_F32
    /* node positions in FP64 for the wall law: origin + anchor + edges */
    double xn[3] = {rv->org[0] + r[0], rv->org[1] + r[1], rv->org[2] + r[2]};
#endif
    for (int j = 0; j <= n; ++j) {
        real mass = 0.0;
        if (j > 0) mass += 0.5 * rv->rho * c->A * rv->lh[j - 1];
        if (j < n) mass += 0.5 * rv->rho * c->A * rv->lh[j];
        double fw[3] = {0.0, 0.0, 0.0};
#ifdef ORC_F32
        if (rv->n_walls) {
            const double vd[3] = {v[3 * j], v[3 * j + 1], v[3 * j + 2]};
            wall_force(rv, xn, vd, fw);
        }
        if (j < n)
            for (int a = 0; a < 3; ++a) xn[a] += r[3 * (j + 1) + a];
#else
        if (rv->n_walls) wall_force(rv, &r[3 * j], &v[3 * j], fw);
#endif
        for (int a = 0; a < 3; ++a) {
            real F = 0.0;
            if (j < n) F += w->nint[3 * j + a];
            if (j > 0) F -= w->nint[3 * (j - 1) + a];
            if (rv->fext) F += rv->fext[3 * j + a];
            if (rv->fconn) F += (real)rv->fconn[3 * j + a];
            F += (real)fw[a];
            F += mass * (real)rv->grav[a];
            acc[3 * j + a] = F / mass - rv->gamma * v[3 * j + a];
        }
    }

    /* elements: Eq. 1b */
    real s_t = 0.0;
    if (rv->camp) s_t = (real)sin(ORC_TWO_PI * rv->freq * t + rv->phase);
    /* homogeneous lab field at time t (Methods, "Magnetized filaments") */
    real bfield[3] = {0.0, 0.0, 0.0};
    if (rv->mag) {
        const double cb = cos(ORC_TWO_PI * rv->field_freq * t), sb = sin(ORC_TWO_PI * rv->field_freq * t);
        for (int a = 0; a < 3; ++a)
            bfield[a] = (real)(rv->field[a] + rv->field[3 + a] * cb + rv->field[6 + a] * sb);
    }
    for (int i = 0; i < n; ++i) {
        const real *Qi = &Q[9 * i];
        const real *wi = &om[3 * i];
        real lh = rv->lh[i], e = w->e[i];
        real J[3] = {rv->rho * c->I1 * lh, rv->rho * c->I2 * lh, rv->rho * c->I3 * lh};
        real tau[3] = {0.0, 0.0, 0.0};
        /* d/ds(B kappa / e^3): difference of Voronoi moments */
        if (rv->drop != 1)
            for (int a = 0; a < 3; ++a) {
                if (i < n - 1) tau[a] += w->M[3 * i + a];
                if (i > 0) tau[a] -= w->M[3 * (i - 1) + a];
            }
        /* kappa x B kappa / e^3: average of the two adjacent Voronoi terms */
        if (rv->drop != 2)
            for (int a = 0; a < 3; ++a) {
                real ysum = 0.0;
                if (i > 0) ysum += w->y[3 * (i - 1) + a];
                if (i < n - 1) ysum += w->y[3 * i + a];
                tau[a] += 0.5 * ysum;
            }
        /* Q t x S sigma, per element (times the rest length) */
        if (rv->drop != 3) {
            real qt[3], sh[3];
            matvec(Qi, &w->t[3 * i], qt);
            cross3(qt, &w->Ssig[3 * i], sh);
            for (int a = 0; a < 3; ++a) tau[a] += sh[a] * lh;
        }
        /* (rho I omega / e) x omega */
        real Jw_e[3] = {J[0] * wi[0] / e, J[1] * wi[1] / e, J[2] * wi[2] / e};
        if (rv->drop != 4) {
            real lt[3];
            cross3(Jw_e, wi, lt);
            for (int a = 0; a < 3; ++a) tau[a] += lt[a];
        }
        /* (rho I omega / e^2) de/dt */
        if (rv->drop != 5)
            for (int a = 0; a < 3; ++a) tau[a] += Jw_e[a] / e * w->edot[i];
        /* external couple per unit length */
        if (rv->camp)
            for (int a = 0; a < 3; ++a) tau[a] += rv->camp[3 * i + a] * s_t * lh;
        /* magnetic couple per unit length, m x (Q b(t)), in the material frame */
        if (rv->mag) {
            real qb[3], cm[3];
            matvec(Qi, bfield, qb);
            cross3(&rv->mag[3 * i], qb, cm);
            for (int a = 0; a < 3; ++a) tau[a] += cm[a] * lh;
        }
        for (int a = 0; a < 3; ++a)
            alpha[3 * i + a] = e * tau[a] / J[a] - rv->gamma * wi[a];
    }
}

static void rod_constraints(const rod_view *rv, real *r, real *v, real *Q, real *om)
{
    const int n = rv->n;
    if (rv->clamp0) {
#ifdef ORC_F32
        /* the anchor: node 0 relative to the origin */
        for (int a = 0; a < 3; ++a) { r[a] = (real)(rv->r0[a] - rv->org[a]); v[a] = 0.0; om[a] = 0.0; }
#else
        for (int a = 0; a < 3; ++a) { r[a] = rv->r0[a]; v[a] = 0.0; om[a] = 0.0; }
#endif
        for (int a = 0; a < 9; ++a) Q[a] = rv->Q0[a];
    }
    if (rv->clamp1) {
#ifdef ORC_F32
        /* the last edge puts node n at its initial position */
        double x[3] = {rv->org[0] + r[0], rv->org[1] + r[1], rv->org[2] + r[2]};
        for (int i = 0; i + 1 < n; ++i)
            for (int a = 0; a < 3; ++a) x[a] += r[3 * (i + 1) + a];
        for (int a = 0; a < 3; ++a) r[3 * n + a] = (real)(rv->r0[3 * n + a] - x[a]);
#endif
        for (int a = 0; a < 3; ++a) {
#ifndef ORC_F32
            r[3 * n + a] = rv->r0[3 * n + a];
#endif
            v[3 * n + a] = 0.0;
            om[3 * (n - 1) + a] = 0.0;
        }
        for (int a = 0; a < 9; ++a) Q[9 * (n - 1) + a] = rv->Q0[9 * (n - 1) + a];
    }
}

static void rod_half_drift(const rod_view *rv, real h, real *r, const real *v, real *Q,
                           const real *om)
{
    const int n = rv->n;
#ifdef ORC_F32
    /* edge form: anchor += h/2 v_0, edge i += h/2 (v_{i+1} - v_i) */
    for (int a = 0; a < 3; ++a) r[a] += 0.5 * h * v[a];
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) r[3 * (i + 1) + a] += 0.5 * h * (v[3 * (i + 1) + a] - v[3 * i + a]);
#else
    for (int j = 0; j <= n; ++j)
        for (int a = 0; a < 3; ++a) r[3 * j + a] += 0.5 * h * v[3 * j + a];
#endif
    for (int i = 0; i < n; ++i) {
        real u[3] = {-0.5 * h * om[3 * i + 0], -0.5 * h * om[3 * i + 1], -0.5 * h * om[3 * i + 2]};
        real E[9], Qn[9];
        rodrigues(u, E);
        mat_ab(E, &Q[9 * i], Qn);
        memcpy(&Q[9 * i], Qn, sizeof Qn);
    }
}

static void rod_steps(const rod_view *rv, double dt, double t0, int64_t step0, int64_t nsteps,
                      real *r, real *v, real *Q, real *om, rod_work *w, real *acc,
                      real *alpha)
{
    rod_consts c;
    rod_consts_make(rv, &c);
    const int n = rv->n;
    const real h = (real)dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        double t_mid = t0 + ((double)(step0 + s) + 0.5) * dt;
        rod_half_drift(rv, h, r, v, Q, om);
        rod_constraints(rv, r, v, Q, om);
        rod_accel(rv, &c, r, v, Q, om, t_mid, w, acc, alpha);
        for (int j = 0; j <= n; ++j)
            for (int a = 0; a < 3; ++a) v[3 * j + a] += h * acc[3 * j + a];
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) om[3 * i + a] += h * alpha[3 * i + a];
        rod_constraints(rv, r, v, Q, om);
        rod_half_drift(rv, h, r, v, Q, om);
        rod_constraints(rv, r, v, Q, om);
    }
}

/* ------------------------------------------------------------------ API */

static int max_elems(const orc_rods *p)
{
    int m = 0;
    for (int r = 0; r < p->n_rods; ++r)
        if (p->n_elems[r] > m) m = p->n_elems[r];
    return m;
}

static void offsets(const orc_rods *p, int64_t *eo, int64_t *no, int64_t *vo)
{
    int64_t e = 0;
    for (int r = 0; r < p->n_rods; ++r) {
        eo[r] = e;
        no[r] = e + r;
        vo[r] = e - r;
        e += p->n_elems[r];
    }
}

/* Connection forces at the current state: fc [N_n][3] (zeroed here). */
static void conn_forces(const orc_rods *p, const double *pos, const double *vel, double *fc, int64_t Nn)
{
    memset(fc, 0, 3 * (size_t)Nn * sizeof(double));
    for (int32_t c = 0; c < p->n_conn; ++c) {
        const int64_t a = p->conn_node[2 * c], b = p->conn_node[2 * c + 1];
        double d[3], dv[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = pos[3 * b + k] - pos[3 * a + k];
            dv[k] = vel[3 * b + k] - vel[3 * a + k];
        }
        const double l = sqrt(dot3d(d, d));
        if (!(l > 0.0)) continue;   /* coincident nodes: no direction, no force */
        double e[3] = {d[0] / l, d[1] / l, d[2] / l};
        const double mag = p->conn_k[c] * (l - p->conn_rest[c]) + p->conn_c[c] * dot3d(e, dv);
        for (int k = 0; k < 3; ++k) {
            fc[3 * a + k] += mag * e[k];
            fc[3 * b + k] -= mag * e[k];
        }
    }
}

/* Contact force on node a (a sphere of radius ra at xa, velocity va) from
 * node b of another rod: the wall law with the overlap of the two spheres,
 * the normal from b to a and their relative velocity.  Adds to f; returns the
 * overlap (<= 0 without contact). */
static double sphere_force(const orc_rods *p, const double *xa, const double *va, double ra, const double *xb,
                           const double *vb, double rb, double *f)
{
    const double d[3] = {xa[0] - xb[0], xa[1] - xb[1], xa[2] - xb[2]};
    const double dist = sqrt(dot3d(d, d));
    const double delta = ra + rb - dist;
    if (!(delta > 0.0) || !(dist > 0.0)) return delta;   /* coincident centres: no direction */
    const double n[3] = {d[0] / dist, d[1] / dist, d[2] / dist};
    const double vr[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
    const double vn = dot3d(n, vr);
    const double fn = delta * (p->wall_k - p->wall_c * vn);
    if (!(fn > 0.0)) return delta;
    const double vt[3] = {vr[0] - vn * n[0], vr[1] - vn * n[1], vr[2] - vn * n[2]};
    const double speed = sqrt(dot3d(vt, vt));
    const double g = p->wall_mu * fn / (speed > p->wall_vslip ? speed : p->wall_vslip);
    for (int k = 0; k < 3; ++k) f[k] += fn * n[k] - g * vt[k];
    return delta;
}

/* Closest points of the segments p0 + s (p1 - p0) and q0 + t (q1 - q0),
 * s, t in [0, 1] (both of positive length): the minimiser of the convex
 * quadratic |p(s) - q(t)|^2 over the unit square.  The unconstrained
 * stationary point's s is clamped to [0, 1], t is the best t for that s,
 * clamped, and when that clamp acts s is re-solved for the clamped t; for
 * parallel segments (no unique stationary point) s starts at 0. */
static void segment_closest(const double *p0, const double *p1, const double *q0, const double *q1, double *s,
                            double *t)
{
    const double d1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double d2[3] = {q1[0] - q0[0], q1[1] - q0[1], q1[2] - q0[2]};
    const double r[3] = {p0[0] - q0[0], p0[1] - q0[1], p0[2] - q0[2]};
    const double a = dot3d(d1, d1), e = dot3d(d2, d2), b = dot3d(d1, d2);
    const double c = dot3d(d1, r), f = dot3d(d2, r);
    const double den = a * e - b * b;   /* >= 0; 0 for parallel segments */
    double ss = 0.0;
    if (den > 1e-12 * a * e) {
        ss = (b * f - c * e) / den;
        ss = ss < 0.0 ? 0.0 : (ss > 1.0 ? 1.0 : ss);
    }
    double tt = (b * ss + f) / e;
    if (tt < 0.0) {
        tt = 0.0;
        ss = -c / a;
        ss = ss < 0.0 ? 0.0 : (ss > 1.0 ? 1.0 : ss);
    } else if (tt > 1.0) {
        tt = 1.0;
        ss = (b - c) / a;
        ss = ss < 0.0 ? 0.0 : (ss > 1.0 ? 1.0 : ss);
    }
    *s = ss;
    *t = tt;
}

/* Exported for the tests: out[0] = s, out[1] = t of segment_closest. */
void orc_segment_closest(const double *p0, const double *p1, const double *q0, const double *q1, double *out)
{
    segment_closest(p0, p1, q0, q1, &out[0], &out[1]);
}

/* Elements i < j of rod r touch each other only when the rest lengths of the
 * elements strictly between them add up to at least the rod's diameter. */
static int self_pair_allowed(const orc_rods *p, const int64_t *eo, int r, int i, int j)
{
    if (j < i) { const int k = i; i = j; j = k; }
    if (j - i < 2) return 0;
    double gap = 0.0;
    for (int k = i + 1; k < j; ++k) gap += (double)p->rest_length[eo[r] + k];
    return gap >= 2.0 * (double)p->radius[r];
}

/* Capsule contact (rod_contact = 2) at the current state, brute force over
 * every ordered pair of elements (element a of rod ra against element b of
 * rod rb): the force on element a goes to its nodes as (1 - s) and s; with pot
 * a quarter of k delta^2 per ordered pair to rod ra.  Each pair's closest
 * points and force are evaluated in one fixed order, the element first in
 * (rod, element) order taking the part of a, and the other element receives
 * the exact negative: the closest-point routine is not symmetric in rounding
 * (nor in its choice for parallel segments), and the two elements of a pair
 * must feel opposite forces for momentum to be conserved. */
static void segment_contact_forces(const orc_rods *p, const double *pos, const double *vel, double *fc,
                                   const int64_t *no, double *pot)
{
    const int R = p->n_rods;
    int64_t *eo = malloc((size_t)R * sizeof(int64_t));
    if (!eo) return;
    int64_t e = 0;
    for (int r = 0; r < R; ++r) {
        eo[r] = e;
        e += p->n_elems[r];
    }
    for (int ra = 0; ra < R; ++ra)
        for (int i = 0; i < p->n_elems[ra]; ++i) {
            const int64_t a0 = no[ra] + i, a1 = a0 + 1;
            double f0[3] = {0.0, 0.0, 0.0}, f1[3] = {0.0, 0.0, 0.0};
            for (int rb = 0; rb < R; ++rb)
                for (int j = 0; j < p->n_elems[rb]; ++j) {
                    if (rb == ra && !self_pair_allowed(p, eo, ra, i, j)) continue;
                    const int64_t b0 = no[rb] + j, b1 = b0 + 1;
                    /* u: the pair's first element in (rod, element) order, w the other */
                    const int a_first = ra < rb || (ra == rb && i < j);
                    const int64_t u0 = a_first ? a0 : b0, u1 = u0 + 1, w0 = a_first ? b0 : a0, w1 = w0 + 1;
                    const double ru = p->radius[a_first ? ra : rb], rw = p->radius[a_first ? rb : ra];
                    double su, sw;
                    segment_closest(&pos[3 * u0], &pos[3 * u1], &pos[3 * w0], &pos[3 * w1], &su, &sw);
                    double xu[3], xw[3], vu[3], vw[3], f[3] = {0.0, 0.0, 0.0};
                    for (int k = 0; k < 3; ++k) {
                        xu[k] = pos[3 * u0 + k] + su * (pos[3 * u1 + k] - pos[3 * u0 + k]);
                        xw[k] = pos[3 * w0 + k] + sw * (pos[3 * w1 + k] - pos[3 * w0 + k]);
                        vu[k] = (1.0 - su) * vel[3 * u0 + k] + su * vel[3 * u1 + k];
                        vw[k] = (1.0 - sw) * vel[3 * w0 + k] + sw * vel[3 * w1 + k];
                    }
                    const double delta = sphere_force(p, xu, vu, ru, xw, vw, rw, f);   /* force on u */
                    if (pot && delta > 0.0) pot[ra] += 0.25 * p->wall_k * delta * delta;
                    const double s = a_first ? su : sw;
                    if (!a_first)
                        for (int k = 0; k < 3; ++k) f[k] = -f[k];
                    for (int k = 0; k < 3; ++k) {
                        f0[k] += (1.0 - s) * f[k];
                        f1[k] += s * f[k];
                    }
                }
            if (fc)
                for (int k = 0; k < 3; ++k) {
                    fc[3 * a0 + k] += f0[k];
                    fc[3 * a1 + k] += f1[k];
                }
        }
    free(eo);
}

/* Rod-rod contact forces at the current state, added to fc [N_n][3] (if
 * non-NULL): every ordered pair of nodes of different rods, by brute force
 * (capsule contact between elements when rod_contact = 2).  With pot
 * (non-NULL, [R]) adds a quarter of k delta^2 per ordered pair to the first
 * node's rod (half of each pair's potential to each rod). */
static void contact_forces(const orc_rods *p, const double *pos, const double *vel, double *fc,
                           const int64_t *no, double *pot)
{
    if (p->rod_contact == 2) {
        segment_contact_forces(p, pos, vel, fc, no, pot);
        return;
    }
    const int R = p->n_rods;
    for (int ra = 0; ra < R; ++ra)
        for (int i = 0; i <= p->n_elems[ra]; ++i) {
            const int64_t a = no[ra] + i;
            double f[3] = {0.0, 0.0, 0.0};
            for (int rb = 0; rb < R; ++rb) {
                if (rb == ra) continue;
                for (int j = 0; j <= p->n_elems[rb]; ++j) {
                    const int64_t b = no[rb] + j;
                    const double delta = sphere_force(p, &pos[3 * a], &vel[3 * a], p->radius[ra], &pos[3 * b],
                                                      &vel[3 * b], p->radius[rb], f);
                    if (pot && delta > 0.0) pot[ra] += 0.25 * p->wall_k * delta * delta;
                }
            }
            if (fc)
                for (int k = 0; k < 3; ++k) fc[3 * a + k] += f[k];
        }
}

/* All rods together, one step at a time (rods joined by connections or in
 * contact). */
static int orc_step_coupled(const orc_rods *p, real *pos, real *vel, real *dir, real *omega,
                            int64_t step0, int64_t n_steps, const int64_t *eo, const int64_t *no,
                            const int64_t *vo)
{
    const int R = p->n_rods;
    const int64_t Nn = no[R - 1] + p->n_elems[R - 1] + 1;
    const int nmax = max_elems(p);
    double *fc = malloc(3 * (size_t)Nn * sizeof(double));
    real *acc = malloc(3 * (size_t)(nmax + 1) * sizeof(real));
    real *alpha = malloc(3 * (size_t)nmax * sizeof(real));
#ifdef ORC_F32
    /* node positions (origin + anchor + edges) and velocities in FP64 for the
     * interaction laws */
    double *xabs = malloc(3 * (size_t)Nn * sizeof(double));
    double *vabs = malloc(3 * (size_t)Nn * sizeof(double));
    rod_work w;
    int fail = (!fc || !acc || !alpha || !xabs || !vabs || work_alloc(&w, nmax) != 0);
#else
    rod_work w;
    int fail = (!fc || !acc || !alpha || work_alloc(&w, nmax) != 0);
#endif
    if (!fail) {
        const double dt = p->dt;
        const real h = (real)dt;
        for (int64_t s = 0; s < n_steps; ++s) {
            const double t_mid = p->t0 + ((double)(step0 + s) + 0.5) * dt;
            for (int r = 0; r < R; ++r) {
                rod_view rv;
                rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
                real *x = pos + 3 * no[r], *v = vel + 3 * no[r], *Q = dir + 9 * eo[r], *om = omega + 3 * eo[r];
                rod_half_drift(&rv, h, x, v, Q, om);
                rod_constraints(&rv, x, v, Q, om);
            }
#ifdef ORC_F32
            for (int r = 0; r < R; ++r) {
                const real *x = pos + 3 * no[r];
                double acc_x[3] = {p->origin[3 * r] + x[0], p->origin[3 * r + 1] + x[1], p->origin[3 * r + 2] + x[2]};
                for (int j = 0; j <= p->n_elems[r]; ++j) {
                    if (j > 0)
                        for (int a = 0; a < 3; ++a) acc_x[a] += x[3 * j + a];
                    for (int a = 0; a < 3; ++a) {
                        xabs[3 * (no[r] + j) + a] = acc_x[a];
                        vabs[3 * (no[r] + j) + a] = vel[3 * (no[r] + j) + a];
                    }
                }
            }
            conn_forces(p, xabs, vabs, fc, Nn);
            if (p->rod_contact) contact_forces(p, xabs, vabs, fc, no, NULL);
#else
            conn_forces(p, pos, vel, fc, Nn);
            if (p->rod_contact) contact_forces(p, pos, vel, fc, no, NULL);
#endif
            for (int r = 0; r < R; ++r) {
                rod_view rv;
                rod_consts c;
                rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
                rod_consts_make(&rv, &c);
                rv.fconn = fc + 3 * no[r];
                const int n = rv.n;
                real *x = pos + 3 * no[r], *v = vel + 3 * no[r], *Q = dir + 9 * eo[r], *om = omega + 3 * eo[r];
                rod_accel(&rv, &c, x, v, Q, om, t_mid, &w, acc, alpha);
                for (int j = 0; j <= n; ++j)
                    for (int a = 0; a < 3; ++a) v[3 * j + a] += h * acc[3 * j + a];
                for (int i = 0; i < n; ++i)
                    for (int a = 0; a < 3; ++a) om[3 * i + a] += h * alpha[3 * i + a];
                rod_constraints(&rv, x, v, Q, om);
                rod_half_drift(&rv, h, x, v, Q, om);
                rod_constraints(&rv, x, v, Q, om);
            }
        }
    }
#ifdef ORC_F32
    if (fc && acc && alpha && xabs && vabs) work_free(&w);   /* work_alloc ran */
    free(xabs);
    free(vabs);
#else
    if (fc && acc && alpha) work_free(&w);   /* work_alloc ran */
#endif
    free(fc);
    free(acc);
    free(alpha);
    return fail ? -2 : 0;
}

/* Advance every rod by n_steps position-Verlet steps, starting at step index
 * step0 (time t0 + step0*dt).  pos/vel [N_n][3], dir [N_e][9], omega [N_e][3]
 * are updated in place.  n_threads <= 0 uses the OpenMP default. */
int orc_step(const orc_rods *p, real *pos, real *vel, real *dir, real *omega,
             int64_t step0, int64_t n_steps, int n_threads)
{
    const int R = p->n_rods;
    if (R <= 0) return 0;
    int64_t *eo = malloc(3 * (size_t)R * sizeof(int64_t));
    if (!eo) return -2;
    int64_t *no = eo + R, *vo = eo + 2 * R;
    offsets(p, eo, no, vo);
    if (p->n_conn > 0 || p->rod_contact) {
        const int rc = orc_step_coupled(p, pos, vel, dir, omega, step0, n_steps, eo, no, vo);
        free(eo);
        return rc;
    }
    const int nmax = max_elems(p);
    int fail = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel reduction(| : fail)
#endif
    {
        rod_work w;
        real *acc = malloc(3 * (size_t)(nmax + 1) * sizeof(real));
        real *alpha = malloc(3 * (size_t)nmax * sizeof(real));
        if (work_alloc(&w, nmax) != 0 || !acc || !alpha) {
            fail = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
            for (int r = 0; r < R; ++r) {
                rod_view rv;
                rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
                rod_steps(&rv, p->dt, p->t0, step0, n_steps, pos + 3 * no[r], vel + 3 * no[r],
                          dir + 9 * eo[r], omega + 3 * eo[r], &w, acc, alpha);
            }
        }
        work_free(&w);
        free(acc);
        free(alpha);
    }
    free(eo);
    return fail ? -2 : 0;
}

#ifndef ORC_F32
/* Strains at a state: sigma [N_e][3], kappa [N_v][3], dilatation e [N_e]. */
int orc_strains(const orc_rods *p, const double *pos, const double *dir, double *sigma,
                double *kappa, double *dil)
{
    const int R = p->n_rods;
    int64_t *eo = malloc(3 * (size_t)R * sizeof(int64_t));
    if (!eo) return -2;
    int64_t *no = eo + R, *vo = eo + 2 * R;
    offsets(p, eo, no, vo);
    rod_work w;
    if (work_alloc(&w, max_elems(p)) != 0) { free(eo); return -2; }
    for (int r = 0; r < R; ++r) {
        rod_view rv;
        rod_consts c;
        rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
        rod_consts_make(&rv, &c);
        rod_kinematics(&rv, &c, pos + 3 * no[r], NULL, dir + 9 * eo[r], &w);
        memcpy(sigma + 3 * eo[r], w.sig, 3 * (size_t)rv.n * sizeof(double));
        memcpy(kappa + 3 * vo[r], w.kap, 3 * (size_t)(rv.n - 1) * sizeof(double));
        if (dil) memcpy(dil + eo[r], w.e, (size_t)rv.n * sizeof(double));
    }
    work_free(&w);
    free(eo);
    return 0;
}

/* Accelerations at a state and time t: acc [N_n][3] (lab), alpha [N_e][3]
 * (material frame), without constraints. */
int orc_accel(const orc_rods *p, const double *pos, const double *vel, const double *dir,
              const double *omega, double t, double *acc, double *alpha)
{
    const int R = p->n_rods;
    int64_t *eo = malloc(3 * (size_t)R * sizeof(int64_t));
    if (!eo) return -2;
    int64_t *no = eo + R, *vo = eo + 2 * R;
    offsets(p, eo, no, vo);
    rod_work w;
    if (work_alloc(&w, max_elems(p)) != 0) { free(eo); return -2; }
    for (int r = 0; r < R; ++r) {
        rod_view rv;
        rod_consts c;
        rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
        rod_consts_make(&rv, &c);
        rod_accel(&rv, &c, pos + 3 * no[r], vel + 3 * no[r], dir + 9 * eo[r], omega + 3 * eo[r],
                  t, &w, acc + 3 * no[r], alpha + 3 * eo[r]);
    }
    work_free(&w);
    free(eo);
    return 0;
}

/* Energies per rod, out [R][5]:
 *   T_lin   = 1/2 sum_j m_j |v_j|^2
 *   T_rot   = 1/2 sum_i omega_i . J_i omega_i / e_i   (angular momentum density rho I omega / e)
 *   U_shear = 1/2 sum_i sigma_i . S sigma_i lh_i
 *   U_bend  = 1/2 sum_k (kappa_k - kappa0_k) . Bv_k (kappa_k - kappa0_k) Dh_k
 *   W_ext   = -sum_j (f_j + m_j g) . (r_j - r_j(0))      (constant nodal forces, gravity) */
int orc_energy(const orc_rods *p, const double *pos, const double *vel, const double *dir,
               const double *omega, double *out)
{
    const int R = p->n_rods;
    int64_t *eo = malloc(3 * (size_t)R * sizeof(int64_t));
    if (!eo) return -2;
    int64_t *no = eo + R, *vo = eo + 2 * R;
    offsets(p, eo, no, vo);
    rod_work w;
    if (work_alloc(&w, max_elems(p)) != 0) { free(eo); return -2; }
    for (int r = 0; r < R; ++r) {
        rod_view rv;
        rod_consts c;
        rod_view_make(p, r, eo[r], no[r], vo[r], &rv);
        rod_consts_make(&rv, &c);
        const int n = rv.n;
        const double *x = pos + 3 * no[r], *v = vel + 3 * no[r], *om = omega + 3 * eo[r];
        rod_kinematics(&rv, &c, x, v, dir + 9 * eo[r], &w);
        double Tl = 0.0, Tr = 0.0, Us = 0.0, Ub = 0.0, Wx = 0.0;
        for (int j = 0; j <= n; ++j) {
            double mass = 0.0;
            if (j > 0) mass += 0.5 * rv.rho * c.A * rv.lh[j - 1];
            if (j < n) mass += 0.5 * rv.rho * c.A * rv.lh[j];
            Tl += 0.5 * mass * dot3(&v[3 * j], &v[3 * j]);
            double d[3] = {x[3 * j] - rv.r0[3 * j], x[3 * j + 1] - rv.r0[3 * j + 1],
                           x[3 * j + 2] - rv.r0[3 * j + 2]};
            if (rv.fext) Wx -= dot3(&rv.fext[3 * j], d);
            Wx -= mass * dot3(rv.grav, d);
            if (rv.n_walls) {
                double fw[3] = {0.0, 0.0, 0.0};
                Wx += wall_force(&rv, &x[3 * j], &v[3 * j], fw);
            }
        }
        for (int i = 0; i < n; ++i) {
            double lh = rv.lh[i];
            double J[3] = {rv.rho * c.I1 * lh, rv.rho * c.I2 * lh, rv.rho * c.I3 * lh};
            for (int a = 0; a < 3; ++a) {
                Tr += 0.5 * om[3 * i + a] * J[a] * om[3 * i + a] / w.e[i];
                Us += 0.5 * w.sig[3 * i + a] * c.S[a] * w.sig[3 * i + a] * lh;
            }
        }
        for (int k = 0; k + 1 < n; ++k) {
            double Dh = 0.5 * (rv.lh[k] + rv.lh[k + 1]);
            for (int a = 0; a < 3; ++a) {
                double Bv = (c.B[a] * rv.lh[k] + c.B[a] * rv.lh[k + 1]) / (rv.lh[k] + rv.lh[k + 1]);
                double dk = w.kap[3 * k + a] - (rv.k0 ? rv.k0[3 * k + a] : 0.0);
                Ub += 0.5 * dk * Bv * dk * Dh;
            }
        }
        out[5 * r + 0] = Tl;
        out[5 * r + 1] = Tr;
        out[5 * r + 2] = Us;
        out[5 * r + 3] = Ub;
        out[5 * r + 4] = Wx;
    }
    /* connection springs: half of each potential to each of the two rods */
    for (int32_t c = 0; c < p->n_conn; ++c) {
        const int64_t a = p->conn_node[2 * c], b = p->conn_node[2 * c + 1];
        double d[3] = {pos[3 * b] - pos[3 * a], pos[3 * b + 1] - pos[3 * a + 1], pos[3 * b + 2] - pos[3 * a + 2]};
        const double ext = sqrt(dot3(d, d)) - p->conn_rest[c];
        const double half = 0.25 * p->conn_k[c] * ext * ext;
        for (int end = 0; end < 2; ++end) {
            const int64_t node = p->conn_node[2 * c + end];
            int r = 0;
            while (r + 1 < R && no[r + 1] <= node) ++r;
            out[5 * r + 4] += half;
        }
    }
    if (p->rod_contact) {
        double *pot = calloc((size_t)R, sizeof(double));
        if (!pot) { work_free(&w); free(eo); return -2; }
        contact_forces(p, pos, vel, NULL, no, pot);
        for (int r = 0; r < R; ++r) out[5 * r + 4] += pot[r];
        free(pot);
    }
    work_free(&w);
    free(eo);
    return 0;
}

/* The two rotation maps, exposed for direct checks. */
void orc_rodrigues(const double *u, double *E) { rodrigues(u, E); }
void orc_logmap(const double *R, double *u) { logmap(R, u); }
#endif /* !ORC_F32: the FP32 build exports the step only */

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
