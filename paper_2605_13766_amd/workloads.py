"""Seeded synthetic rod batches.

This module only builds *inputs*: centrelines, director frames, material
parameters, boundary flags and loads, as host FP64 numpy arrays in the layout
of the C boundary (``include/rod.h``).  It contains none of the rod method's
arithmetic (no strains, forces, couples or time stepping), so both the GPU path
and the CPU oracle can consume the very same arrays.

Workloads follow the problem statement of the Cosserat-rod model (Methods,
"Cosserat rod dynamics": centreline r, row director matrix Q = {d1,d2,d3}^T,
material parameters rho, E, G, alpha_c, cross-section) and these batch
shapes:

* ``single_cantilever``  : 1 rod, 100 elements, 1 m, clamped at s=0, tip force.
* ``ragged_batch``       : free-free rods of 16..256 elements, smooth random
  3-mode Fourier centrelines with curvature <= 5/m, log-uniform E.
* ``cilia_carpet``       : base-clamped vertical rods on a square grid, each
  driven by a sinusoidal bending couple with a random phase.
* ``surrogate_training`` : the carpet regime at 64 elements with random couple
  amplitude and velocity noise (training data for the learned coarse step).
* ``magnetic_carpet``    : the carpet driven instead by a rotating homogeneous
  magnetic field acting on a programmed per-rod magnetization (Methods,
  "Magnetized filaments"; Results, "Magnetized filament assemblies").
* ``active_filaments``   : free rods scattered in a box, under gravity and
  driven by travelling-wave muscle moments (Results, "Active matter").

Node j of rod r is row ``node_offset[r] + j`` of the node arrays, element i
is row ``elem_offset[r] + i`` of the element arrays, Voronoi point k is row
``elem_offset[r] - r + k``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

SEED_BASE = 137660

# shear modulus ratio and shear coefficient used by every workload here
G_OVER_E = 1.0 / 1.5
SHEAR_COEFF = 4.0 / 3.0
DENSITY = 1000.0


@dataclasses.dataclass
class RodInputs:
    """One batch of rods in the boundary's layout (all FP64 / int32, host)."""

    n_elems: np.ndarray            # [R] int32
    position: np.ndarray           # [N_n, 3]
    velocity: np.ndarray           # [N_n, 3]
    director: np.ndarray           # [N_e, 3, 3]  rows d1, d2, d3
    omega: np.ndarray              # [N_e, 3]     material frame
    density: np.ndarray            # [R]
    youngs: np.ndarray             # [R]
    shear_modulus: np.ndarray      # [R]
    radius: np.ndarray             # [R]
    shear_coeff: np.ndarray        # [R]
    damping: np.ndarray            # [R]  1/s
    bc_start: np.ndarray           # [R] int32, 1 = clamped at s=0
    bc_end: np.ndarray             # [R] int32, 1 = clamped at s=L
    dt: float
    rest_length: Optional[np.ndarray] = None   # [N_e] or None -> from position
    rest_kappa: Optional[np.ndarray] = None    # [N_v, 3] or None -> 0
    end_force: Optional[np.ndarray] = None     # [R, 3] on the last node
    couple_amp: Optional[np.ndarray] = None    # [R, 3] per unit length, material frame
    couple_freq: Optional[np.ndarray] = None   # [R] Hz
    couple_phase: Optional[np.ndarray] = None  # [R] rad
    magnetization: Optional[np.ndarray] = None  # [N_e, 3] per unit length, material frame (A m)
    field: Optional[np.ndarray] = None          # [9]: b(t) = f[0:3] + f[3:6] cos(2 pi ff t) + f[6:9] sin(...), T
    field_freq: float = 0.0                     # ff, Hz
    gravity: Optional[np.ndarray] = None        # [3] m/s^2, lab frame
    muscle_amp: Optional[np.ndarray] = None     # [N_v] N m: beta_k at Voronoi point k
    muscle_axis: Optional[np.ndarray] = None    # [R, 3] material frame
    muscle_freq: Optional[np.ndarray] = None    # [R] Hz
    muscle_wavenumber: Optional[np.ndarray] = None  # [R] rad/m
    muscle_phase: Optional[np.ndarray] = None   # [R] rad
    conn_rod: Optional[np.ndarray] = None       # [C, 2] int32: rods of the two connected nodes
    conn_node: Optional[np.ndarray] = None      # [C, 2] int32: node index within each rod (0..n)
    conn_k: Optional[np.ndarray] = None         # [C] N/m
    conn_c: Optional[np.ndarray] = None         # [C] N s/m
    conn_rest: Optional[np.ndarray] = None      # [C] m
    walls: Optional[np.ndarray] = None          # [n_walls, 4]: unit normal, offset (wall n.x = d)
    wall_k: float = 0.0                         # N/m
    wall_c: float = 0.0                         # N s/m^2 (damping per unit penetration)
    wall_mu: float = 0.0
    wall_vslip: float = 1e-4                    # m/s
    rod_contact: int = 0                        # 1: nodes of different rods touch (spheres, the wall law); 2: elements (capsules)
    name: str = ""

    # ------------------------------------------------------------------ sizes
    @property
    def n_rods(self) -> int:
        return int(self.n_elems.shape[0])

    @property
    def n_elements(self) -> int:
        return int(self.n_elems.sum())

    @property
    def elem_offset(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.n_elems)[:-1]]).astype(np.int64)

    @property
    def node_offset(self) -> np.ndarray:
        return self.elem_offset + np.arange(self.n_rods, dtype=np.int64)

    @property
    def vor_offset(self) -> np.ndarray:
        return self.elem_offset - np.arange(self.n_rods, dtype=np.int64)

    def copy(self) -> "RodInputs":
        kw = {}
        for f in dataclasses.fields(self):
            v = getattr(self, f.name)
            kw[f.name] = v.copy() if isinstance(v, np.ndarray) else v
        return RodInputs(**kw)

    def subset(self, rods) -> "RodInputs":
        """A new batch holding only the listed rods (in the given order)."""
        rods = np.asarray(rods, dtype=np.int64)
        eo, no, vo = self.elem_offset, self.node_offset, self.vor_offset
        n = self.n_elems
        e_idx = np.concatenate([np.arange(eo[r], eo[r] + n[r]) for r in rods])
        n_idx = np.concatenate([np.arange(no[r], no[r] + n[r] + 1) for r in rods])
        v_idx = np.concatenate([np.arange(vo[r], vo[r] + n[r] - 1) for r in rods])

        def per_rod(a):
            return None if a is None else a[rods].copy()

        return RodInputs(
            n_elems=n[rods].copy(),
            position=self.position[n_idx].copy(),
            velocity=self.velocity[n_idx].copy(),
            director=self.director[e_idx].copy(),
            omega=self.omega[e_idx].copy(),
            density=per_rod(self.density), youngs=per_rod(self.youngs),
            shear_modulus=per_rod(self.shear_modulus), radius=per_rod(self.radius),
            shear_coeff=per_rod(self.shear_coeff), damping=per_rod(self.damping),
            bc_start=per_rod(self.bc_start), bc_end=per_rod(self.bc_end),
            dt=self.dt,
            rest_length=None if self.rest_length is None else self.rest_length[e_idx].copy(),
            rest_kappa=None if self.rest_kappa is None else self.rest_kappa[v_idx].copy(),
            end_force=per_rod(self.end_force), couple_amp=per_rod(self.couple_amp),
            couple_freq=per_rod(self.couple_freq), couple_phase=per_rod(self.couple_phase),
            magnetization=None if self.magnetization is None else self.magnetization[e_idx].copy(),
            field=None if self.field is None else np.array(self.field, float).copy(),
            field_freq=self.field_freq,
            gravity=None if self.gravity is None else np.array(self.gravity, float).copy(),
            muscle_amp=None if self.muscle_amp is None else self.muscle_amp[v_idx].copy(),
            muscle_axis=per_rod(self.muscle_axis), muscle_freq=per_rod(self.muscle_freq),
            muscle_wavenumber=per_rod(self.muscle_wavenumber), muscle_phase=per_rod(self.muscle_phase),
            **self._subset_connections(rods),
            walls=None if self.walls is None else np.array(self.walls, float).copy(),
            wall_k=self.wall_k, wall_c=self.wall_c, wall_mu=self.wall_mu, wall_vslip=self.wall_vslip,
            rod_contact=self.rod_contact, name=self.name + "[subset]",
        )

    def _subset_connections(self, rods):
        """Connections whose two rods are both in `rods`, renumbered."""
        if self.conn_rod is None:
            return {}
        where = {int(r): k for k, r in enumerate(rods)}
        keep = [c for c in range(len(self.conn_rod))
                if int(self.conn_rod[c, 0]) in where and int(self.conn_rod[c, 1]) in where]
        if not keep:
            return {}
        cr = np.array([[where[int(self.conn_rod[c, 0])], where[int(self.conn_rod[c, 1])]] for c in keep], np.int32)
        return dict(conn_rod=cr, conn_node=self.conn_node[keep].copy(), conn_k=self.conn_k[keep].copy(),
                    conn_c=self.conn_c[keep].copy(), conn_rest=self.conn_rest[keep].copy())


# ---------------------------------------------------------------------------
# geometry helpers (frames for given centrelines; no mechanics)
# ---------------------------------------------------------------------------

def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _any_perpendicular(d3):
    a = np.array([1.0, 0.0, 0.0]) if abs(d3[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    d1 = a - np.dot(a, d3) * d3
    return d1 / np.linalg.norm(d1)


def _rotate_about(v, axis, angle):
    """Rotate vector v about unit axis by angle (right hand)."""
    c, s = np.cos(angle), np.sin(angle)
    return v * c + np.cross(axis, v) * s + axis * np.dot(axis, v) * (1.0 - c)


def frames_parallel_transport(nodes, d1_first=None):
    """Director rows for the chords of a polyline, d1 carried by parallel transport.

    d3_i is the unit chord of element i; d1 is transported from element to
    element by the smallest rotation taking d3_i onto d3_{i+1}; d2 = d3 x d1.
    Returns [n, 3, 3] with rows d1, d2, d3.
    """
    chords = np.diff(nodes, axis=0)
    d3 = _unit(chords)
    n = d3.shape[0]
    Q = np.empty((n, 3, 3))
    d1 = _any_perpendicular(d3[0]) if d1_first is None else np.asarray(d1_first, float)
    for i in range(n):
        if i > 0:
            axis = np.cross(d3[i - 1], d3[i])
            s = np.linalg.norm(axis)
            if s > 1e-15:
                ang = np.arctan2(s, np.dot(d3[i - 1], d3[i]))
                d1 = _rotate_about(d1, axis / s, ang)
            d1 = d1 - np.dot(d1, d3[i]) * d3[i]
            d1 = d1 / np.linalg.norm(d1)
        d2 = np.cross(d3[i], d1)
        Q[i, 0], Q[i, 1], Q[i, 2] = d1, d2, d3[i]
    return Q


def _fourier_curve(rng, L, n, kappa_max):
    """Nodes of one smooth 3-mode Fourier curve of arclength L, resampled to n
    equal chords, largest curvature below kappa_max (see ``_fourier_curves``)."""
    return _fourier_curves(rng, np.array([float(L)]), np.array([int(n)]), float(kappa_max))[0]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def _assemble(name, nodes_list, Q_list, dt, *, density, youngs, radius, damping,
              bc_start, bc_end, velocity_list=None, omega_list=None,
              end_force=None, couple_amp=None, couple_freq=None, couple_phase=None):
    R = len(nodes_list)
    n_elems = np.array([Q.shape[0] for Q in Q_list], dtype=np.int32)
    position = np.concatenate(nodes_list, axis=0).astype(np.float64)
    director = np.concatenate(Q_list, axis=0).astype(np.float64)
    velocity = (np.zeros_like(position) if velocity_list is None
                else np.concatenate(velocity_list, axis=0).astype(np.float64))
    omega = (np.zeros((director.shape[0], 3)) if omega_list is None
             else np.concatenate(omega_list, axis=0).astype(np.float64))
    f = lambda x: np.array(np.broadcast_to(np.asarray(x, np.float64), (R,)))
    return RodInputs(
        n_elems=n_elems, position=np.ascontiguousarray(position),
        velocity=np.ascontiguousarray(velocity),
        director=np.ascontiguousarray(director), omega=np.ascontiguousarray(omega),
        density=f(density), youngs=f(youngs), shear_modulus=f(np.asarray(youngs) * G_OVER_E),
        radius=f(radius), shear_coeff=f(SHEAR_COEFF), damping=f(damping),
        bc_start=np.array(np.broadcast_to(np.asarray(bc_start, np.int32), (R,))),
        bc_end=np.array(np.broadcast_to(np.asarray(bc_end, np.int32), (R,))),
        dt=float(dt), end_force=end_force, couple_amp=couple_amp,
        couple_freq=couple_freq, couple_phase=couple_phase, name=name)


def straight_rod(n, L, direction=(1.0, 0.0, 0.0), d1=(0.0, 1.0, 0.0), origin=(0.0, 0.0, 0.0)):
    """Nodes and directors of a straight rod (d3 along `direction`)."""
    d3 = _unit(np.asarray(direction, float))
    d1 = np.asarray(d1, float)
    d1 = _unit(d1 - np.dot(d1, d3) * d3)
    d2 = np.cross(d3, d1)
    s = np.linspace(0.0, L, n + 1)
    nodes = np.asarray(origin, float)[None, :] + s[:, None] * d3[None, :]
    Q = np.broadcast_to(np.stack([d1, d2, d3]), (n, 3, 3)).copy()
    return nodes, Q


def single_cantilever(n=100, L=1.0, radius=0.01, youngs=1e6, tip_force=(0.0, 0.0, -1e-3),
                      noise=1e-6, dt=1e-5, seed=SEED_BASE + 1):
    """One rod clamped at s=0 with a constant force on its last node.

    Straight along +x with d1 = y, d2 = z, d3 = x; velocity noise N(0, noise^2)
    on every free node; no damping.
    """
    rng = np.random.default_rng(seed)
    nodes, Q = straight_rod(n, L)
    vel = np.zeros_like(nodes)
    if noise > 0:
        vel[1:] = rng.normal(0.0, noise, size=(n, 3))
    return _assemble("single_cantilever", [nodes], [Q], dt, density=DENSITY, youngs=youngs,
                     radius=radius, damping=0.0, bc_start=1, bc_end=0, velocity_list=[vel],
                     end_force=np.asarray(tip_force, float).reshape(1, 3).copy())


def _fourier_curves(rng, L, ns, kappa_max, samples=257):
    """Batched ``_fourier_curve``: one smooth 3-mode Fourier curve per rod, with
    analytic derivatives for the curvature and a vectorised bisection on the
    perturbation scale; returns a list of [n_r + 1, 3] node arrays.  The scale
    also keeps |r'| >= 1/2 everywhere, so no cusp can hide between samples."""
    R = len(L)
    e = _unit(rng.normal(size=(R, 3)))
    a = rng.normal(size=(R, 3, 3))          # [rod, mode, xyz]
    b = rng.normal(size=(R, 3, 3))
    u = np.linspace(0.0, 1.0, samples)
    k = np.pi * np.arange(1, 4)[:, None]    # m pi
    sp, cp = np.sin(k * u[None, :]), np.cos(k * u[None, :])
    P = np.einsum("rmx,ms->rsx", a, sp) + np.einsum("rmx,ms->rsx", b, 1.0 - cp)
    P1 = (np.einsum("rmx,ms->rsx", a, k * cp) + np.einsum("rmx,ms->rsx", b, k * sp)) / L[:, None, None]
    P2 = (np.einsum("rmx,ms->rsx", a, -k * k * sp) + np.einsum("rmx,ms->rsx", b, k * k * cp)) \
        / (L ** 2)[:, None, None]

    def ok(lam):
        r1 = e[:, None, :] + lam[:, None, None] * P1
        r2 = lam[:, None, None] * P2
        sp1 = np.linalg.norm(r1, axis=2)
        kmax = (np.linalg.norm(np.cross(r1, r2), axis=2) / sp1 ** 3).max(axis=1)
        # stay in the small-perturbation branch: speed within [0.8, 1.2] of the
        # straight line, so the final rescaling to length L changes the
        # curvature by less than 1.2x (budgeted in the bound)
        return (kmax < kappa_max / 1.2) & (sp1.min(axis=1) > 0.8) & (sp1.max(axis=1) < 1.2)

    # curvature is not monotonic in the scale (a huge loop is flat again), so
    # grow from a tiny scale to the first failure, then bisect that interval
    lo = np.zeros(R)
    hi = np.full(R, 1e-6)
    active = np.ones(R, dtype=bool)
    for _ in range(80):
        good = ok(hi) & active
        if not good.any():
            break
        lo = np.where(good, hi, lo)
        hi = np.where(good, hi * 2.0, hi)
        active = good
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        below = ok(mid)
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    curves = u[None, :, None] * L[:, None, None] * e[:, None, :] + lo[:, None, None] * P
    out = []
    for r in range(R):
        c = curves[r]
        seg = np.linalg.norm(np.diff(c, axis=0), axis=1)
        arc = np.concatenate([[0.0], np.cumsum(seg)])
        targ = np.linspace(0.0, arc[-1], int(ns[r]) + 1)
        nodes = np.stack([np.interp(targ, arc, c[:, x]) for x in range(3)], axis=1)
        out.append(nodes * (L[r] / arc[-1]))
    return out


def _frames_batched(nodes_list):
    """``frames_parallel_transport`` for many polylines at once (padded)."""
    R = len(nodes_list)
    ns = np.array([x.shape[0] - 1 for x in nodes_list])
    nmax = ns.max()
    d3 = np.zeros((R, nmax, 3))
    for r, x in enumerate(nodes_list):
        c = _unit(np.diff(x, axis=0))
        d3[r, :ns[r]] = c
        d3[r, ns[r]:] = c[-1]
    Q = np.empty((R, nmax, 3, 3))
    a = np.where(np.abs(d3[:, 0, 0:1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    d1 = _unit(a - np.sum(a * d3[:, 0], axis=1, keepdims=True) * d3[:, 0])
    for i in range(nmax):
        if i > 0:
            axis = np.cross(d3[:, i - 1], d3[:, i])
            sn = np.linalg.norm(axis, axis=1)
            cs = np.sum(d3[:, i - 1] * d3[:, i], axis=1)
            ang = np.arctan2(sn, cs)
            k = axis / np.where(sn > 1e-15, sn, 1.0)[:, None]
            c, s_ = np.cos(ang)[:, None], np.sin(ang)[:, None]
            rot = d1 * c + np.cross(k, d1) * s_ + k * np.sum(k * d1, axis=1, keepdims=True) * (1.0 - c)
            d1 = np.where((sn > 1e-15)[:, None], rot, d1)
            d1 = _unit(d1 - np.sum(d1 * d3[:, i], axis=1, keepdims=True) * d3[:, i])
        Q[:, i, 0] = d1
        Q[:, i, 1] = np.cross(d3[:, i], d1)
        Q[:, i, 2] = d3[:, i]
    return [Q[r, :ns[r]].copy() for r in range(R)]


def ragged_batch(n_rods=4096, n_min=16, n_max=256, ds=0.01, kappa_max=5.0, damping=0.1,
                 dt=1e-5, seed=SEED_BASE + 2, box=5.0):
    """Free-free rods with uneven element counts and curved centrelines.

    Element count uniform in [n_min, n_max]; rod length n*ds; centrelines are
    3-mode Fourier curves whose largest curvature is drawn in [0.2, 0.95] x
    kappa_max; rest state straight and unstretched at the initial chord lengths;
    E log-uniform in [1e5, 1e7] Pa; radius uniform in [0.005, 0.02] m; d1 by
    parallel transport along the chords.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, size=n_rods)
    E = 10.0 ** rng.uniform(5.0, 7.0, size=n_rods)
    rad = rng.uniform(0.005, 0.02, size=n_rods)
    kap = kappa_max * rng.uniform(0.2, 0.95, size=n_rods)
    nodes_list = _fourier_curves(rng, ns * ds, ns, kap)
    base = rng.uniform(-box, box, size=(n_rods, 3))
    nodes_list = [x + base[r][None, :] for r, x in enumerate(nodes_list)]
    Q_list = _frames_batched(nodes_list)
    return _assemble("ragged_batch", nodes_list, Q_list, dt, density=DENSITY, youngs=E,
                     radius=rad, damping=damping, bc_start=0, bc_end=0)


def cilia_carpet(grid=256, n=50, L=0.01, radius=2e-4, youngs=1e6, spacing=2.5e-3,
                 amp=7.5e-6, freq=10.0, dt=1e-6, seed=SEED_BASE + 3, amp_range=None,
                 noise=0.0, n_rods=None):
    """Vertical rods clamped at their base on a grid x grid lattice.

    Each rod carries a distributed couple amp*sin(2 pi freq t + phi) about its
    material d1 axis, with phi uniform in [0, 2 pi).  d1 = x, d2 = y, d3 = z.
    ``amp_range=(lo, hi)`` scales amp per rod by U[lo, hi]; ``noise`` adds
    N(0, noise^2) velocity noise on free nodes; ``n_rods`` truncates the grid.
    """
    rng = np.random.default_rng(seed)
    R = grid * grid if n_rods is None else int(n_rods)
    ix, iy = np.divmod(np.arange(R), grid)
    base = np.stack([ix * spacing, iy * spacing, np.zeros(R)], axis=1)
    s = np.linspace(0.0, L, n + 1)
    nodes = base[:, None, :] + s[None, :, None] * np.array([0.0, 0.0, 1.0])[None, None, :]
    Q1 = np.stack([np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])])
    director = np.broadcast_to(Q1, (R * n, 3, 3)).copy()
    phase = rng.uniform(0.0, 2.0 * np.pi, size=R)
    scale = np.ones(R) if amp_range is None else rng.uniform(amp_range[0], amp_range[1], size=R)
    camp = np.zeros((R, 3))
    camp[:, 0] = amp * scale
    vel = np.zeros((R, n + 1, 3))
    if noise > 0:
        vel[:, 1:, :] = rng.normal(0.0, noise, size=(R, n, 3))
    inp = RodInputs(
        n_elems=np.full(R, n, dtype=np.int32),
        position=np.ascontiguousarray(nodes.reshape(-1, 3)),
        velocity=np.ascontiguousarray(vel.reshape(-1, 3)),
        director=director, omega=np.zeros((R * n, 3)),
        density=np.full(R, DENSITY), youngs=np.full(R, float(youngs)),
        shear_modulus=np.full(R, youngs * G_OVER_E), radius=np.full(R, float(radius)),
        shear_coeff=np.full(R, SHEAR_COEFF), damping=np.zeros(R),
        bc_start=np.ones(R, dtype=np.int32), bc_end=np.zeros(R, dtype=np.int32),
        dt=float(dt), couple_amp=camp, couple_freq=np.full(R, float(freq)),
        couple_phase=phase, name="cilia_carpet")
    return inp


def surrogate_training(n_rods=16384, n=64, seed=SEED_BASE + 4, **kw):
    """Training rods: the carpet regime at 64 elements, random couple amplitude in
    [0.5, 1.5] x 7.5e-6 N m/m and N(0, 1e-6 m/s) velocity noise."""
    grid = int(np.ceil(np.sqrt(n_rods)))
    return cilia_carpet(grid=grid, n=n, seed=seed, amp_range=(0.5, 1.5), noise=1e-6,
                        n_rods=n_rods, **kw)


def surrogate_at_scale(n_rods=262144, n=64, seed=SEED_BASE + 5, **kw):
    """Rods advanced by the learned coarse step: the carpet regime at 64 elements."""
    grid = int(np.ceil(np.sqrt(n_rods)))
    return cilia_carpet(grid=grid, n=n, seed=seed, amp_range=(0.5, 1.5), noise=1e-6,
                        n_rods=n_rods, **kw)


def magnetic_carpet(grid=256, n=50, L=0.01, radius=2e-4, youngs=1e6, spacing=2.5e-3,
                    m0=1.5e-3, b0=0.01, freq=10.0, wavelengths=(16.0, 24.0), dt=1e-6,
                    seed=SEED_BASE + 6, n_rods=None, noise=0.0):
    """The cilia carpet with its driving couple replaced by a magnetic one.

    Every element of the rod at lattice site (ix, iy) carries the magnetization
    per unit length m0 (sin phi, 0, cos phi) in its material frame (d1 = x,
    d3 = z along the rod), phi = 2 pi (ix / lambda_x + iy / lambda_y): the
    programmed profile whose phase lag from rod to rod makes the beats of a
    homogeneous field travel as a metachronal wave, with different wavelengths
    (in lattice spacings) along x and y so that it runs diagonally.  The field
    rotates in the x-z plane, b(t) = b0 (sin 2 pi f t, 0, cos 2 pi f t).
    Defaults: m0 b0 = 1.5e-5 N m/m, twice the driven carpet's couple
    amplitude (a composite magnetization of about 1.2e4 A/m over the
    cross-section); ``noise`` adds N(0, noise^2) velocity noise on free nodes.
    """
    inp = cilia_carpet(grid=grid, n=n, L=L, radius=radius, youngs=youngs, spacing=spacing,
                       dt=dt, seed=seed, noise=noise, n_rods=n_rods)
    R = len(inp.n_elems)
    ix, iy = np.divmod(np.arange(R), grid)
    phi = 2.0 * np.pi * (ix / wavelengths[0] + iy / wavelengths[1])
    m = np.stack([m0 * np.sin(phi), np.zeros(R), m0 * np.cos(phi)], axis=1)
    inp.magnetization = np.ascontiguousarray(np.repeat(m, n, axis=0))
    inp.field = np.array([0.0, 0.0, 0.0, 0.0, 0.0, b0, b0, 0.0, 0.0])
    inp.field_freq = float(freq)
    inp.couple_amp = inp.couple_freq = inp.couple_phase = None
    inp.name = "magnetic_carpet"
    return inp


def active_filaments(n_rods=16384, n=50, L=1.0, radius=0.025, youngs=1e7, period=1.0,
                     wavelength=None, curvature_amp=3.0, g=9.81, damping=0.5, dt=5e-5,
                     seed=SEED_BASE + 7, box=False, wall_k=1e4, wall_c=2e4, wall_mu=0.3, wall_vslip=1e-3):
    """Free straight filaments at random positions and orientations in a cube of
    side 2L, under gravity (-z) and each driven by a travelling muscle wave.

    The muscle moment at Voronoi point k is beta_k sin(2 pi t / period - 2 pi
    s_k / wavelength + phi_r) about the material d1 axis, with
    beta_k = curvature_amp E I sin(pi s_k / L) (the curvature it would hold
    statically, tapered to zero at both ends) and a random phase phi_r per rod;
    wavelength defaults to L.  Defaults follow a snake-sized rod (1 m, radius
    25 mm, E = 1e7 Pa, one wave per second).
    """
    rng = np.random.default_rng(seed)
    wavelength = L if wavelength is None else wavelength
    # with box=True, centres stay within [L/2, 3L/2] so every node starts inside the 2L box
    base = rng.uniform(0.5 * L, 1.5 * L, size=(n_rods, 3)) if box else rng.uniform(0.0, 2.0 * L, size=(n_rods, 3))
    d3 = _unit(rng.normal(size=(n_rods, 3)))
    s = np.linspace(0.0, L, n + 1)
    nodes = base[:, None, :] + (s - 0.5 * L)[None, :, None] * d3[:, None, :]
    a = np.where(np.abs(d3[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    d1 = _unit(a - np.sum(a * d3, axis=1, keepdims=True) * d3)
    d2 = np.cross(d3, d1)
    Q = np.repeat(np.stack([d1, d2, d3], axis=1), n, axis=0)
    inp = _assemble("active_filaments", list(nodes), list(Q.reshape(n_rods, n, 3, 3)), dt,
                    density=DENSITY, youngs=youngs, radius=radius, damping=damping, bc_start=0, bc_end=0)
    EI = youngs * np.pi * radius ** 4 / 4.0
    sk = np.arange(1, n) * (L / n)
    inp.gravity = np.array([0.0, 0.0, -g])
    inp.muscle_amp = np.tile(curvature_amp * EI * np.sin(np.pi * sk / L), n_rods)
    inp.muscle_axis = np.tile([1.0, 0.0, 0.0], (n_rods, 1))
    inp.muscle_freq = np.full(n_rods, 1.0 / period)
    inp.muscle_wavenumber = np.full(n_rods, 2.0 * np.pi / wavelength)
    inp.muscle_phase = rng.uniform(0.0, 2.0 * np.pi, size=n_rods)
    if box:
        # the paper's cuboidal box of side 2L: floor, ceiling and four side walls
        inp.walls = np.array([[0, 0, 1, 0], [0, 0, -1, -2 * L], [1, 0, 0, 0], [-1, 0, 0, -2 * L],
                              [0, 1, 0, 0], [0, -1, 0, -2 * L]], float)
        inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = wall_k, wall_c, wall_mu, wall_vslip
        inp.name = "active_box"
    return inp


def fibre_pile(n_rods=16384, n=50, L=0.5, radius=0.01, youngs=1e7, per_row=8, rows=100, overlap=1e-7,
               g=9.81, damping=0.5, dt=1e-5, contact_k=1e5, contact_c=1e3, mu=0.3, vslip=1e-2, noise=1e-3,
               seed=SEED_BASE + 9, contact=1):
    """Straight fibres in crossed layers on a floor, in rod-rod contact (the
    paper's fibrous granular materials).

    Layer q holds per_row x rows fibres of length L, along x in even layers and
    along y in odd ones, rows 4 radii apart and fibres end to end with a gap of
    4 radii; layers are 2 radii minus `overlap` apart, so every crossing starts
    in light contact, and the lowest layer rests on a floor wall at z = 0.
    Gravity, linear damping, the contact law with stiffness contact_k, damping
    contact_c, friction mu below slip speed vslip; node velocities N(0, noise^2)
    break the lattice's symmetry.  Defaults: 16,384 fibres of 50 elements in
    21 layers of 800 (element length 1 cm = one radius, so a crossing meets
    several nodes of each fibre).  contact=2 makes the elements capsules
    (segment contact, self-contact included) instead of node spheres.
    """
    rng = np.random.default_rng(seed)
    sp = 4.0 * radius
    per_layer = per_row * rows
    nodes_list, Q_list = [], []
    for r in range(n_rods):
        q, k = divmod(r, per_layer)
        j, i = divmod(k, per_row)
        z = radius + q * (2.0 * radius - overlap)
        along, across = i * (L + sp), (j + 0.5) * sp
        if q % 2 == 0:
            nodes, Q = straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(along, across, z))
        else:
            nodes, Q = straight_rod(n, L, direction=(0, 1, 0), d1=(0, 0, 1), origin=(across, along, z))
        nodes_list.append(nodes)
        Q_list.append(Q)
    vel = [rng.normal(0.0, noise, size=(n + 1, 3)) for _ in range(n_rods)]
    inp = _assemble("fibre_pile", nodes_list, Q_list, dt, density=DENSITY, youngs=youngs, radius=radius,
                    damping=damping, bc_start=0, bc_end=0, velocity_list=vel)
    inp.gravity = np.array([0.0, 0.0, -g])
    inp.walls = np.array([[0.0, 0.0, 1.0, 0.0]])
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = contact_k, contact_c, mu, vslip
    inp.rod_contact = contact
    return inp


def capsule_pile(n_rods=16384, n=20, radius=0.01, **kw):
    """The fibre pile with the paper's fibre aspect ratio (length 31 diameters,
    0.62 m at a radius of 1 cm) in capsule contact: n = 20 elements of 3.1
    radii, longer than the diameter, so crossing fibres meet between nodes and
    only segment contact sees them."""
    return fibre_pile(n_rods=n_rods, n=n, L=62.0 * radius, radius=radius, contact=2, seed=SEED_BASE + 10, **kw)


def millipede_swarm(n_bots=224, legs_per_side=12, n_back=20, n_leg=8, back_length=0.02, leg_length=0.004,
                    back_radius=2.5e-4, leg_radius=2e-4, width=2e-3, youngs=1e6, k_lateral=1.0, k_leg=1.0,
                    c_conn=1e-5, m0=1e-4, b0=0.01, freq=5.0, spacing=0.03, dt=1e-6, seed=SEED_BASE + 8):
    """Millipede-like bots of connected rods (Results, "Magnetized filament
    assemblies"): per bot two parallel backbone rods along x, `width` apart,
    joined node by node by lateral connections (distributed connection, rest
    length `width`), and `legs_per_side` legs per backbone, each attached
    point-wise (rest length 0) by its first node to a backbone node and
    pointing outward and down.  The legs carry a magnetization m0 along their
    axis whose sign alternates along the bot; the field rotates in the x-z
    plane.  Bots sit on a square grid `spacing` apart; each bot is one
    connected group (2 * n_back + 2 * legs_per_side * n_leg elements).
    """
    rng = np.random.default_rng(seed)
    g = int(np.ceil(np.sqrt(n_bots)))
    nodes_list, Q_list, radius, rods = [], [], [], []
    conn_rod, conn_node, conn_k, conn_rest = [], [], [], []
    mag = []
    for bot in range(n_bots):
        ox, oy = (bot % g) * spacing, (bot // g) * spacing
        base = np.array([ox, oy, 0.0]) + rng.normal(0, 1e-5, 3)
        first = len(nodes_list)
        for side in (0, 1):
            nodes, Q = straight_rod(n_back, back_length, direction=(1, 0, 0), d1=(0, 0, 1),
                                    origin=base + np.array([0.0, side * width, 0.0]))
            nodes_list.append(nodes); Q_list.append(Q); radius.append(back_radius)
            mag.append(np.zeros((n_back, 3)))
        for j in range(n_back + 1):      # lateral connections, node by node
            conn_rod.append([first, first + 1]); conn_node.append([j, j]); conn_k.append(k_lateral)
            conn_rest.append(width)
        at = np.linspace(1, n_back - 1, legs_per_side).round().astype(int)
        for side in (0, 1):
            out = -1.0 if side == 0 else 1.0
            for li, j in enumerate(at):
                root = nodes_list[first + side][j]
                direction = np.array([0.0, out * np.cos(np.pi / 4), -np.sin(np.pi / 4)])
                nodes, Q = straight_rod(n_leg, leg_length, direction=direction, d1=(1, 0, 0), origin=root)
                nodes_list.append(nodes); Q_list.append(Q); radius.append(leg_radius)
                sign = 1.0 if li % 2 == 0 else -1.0
                mag.append(np.tile([0.0, 0.0, sign * m0], (n_leg, 1)))
                conn_rod.append([first + side, len(nodes_list) - 1]); conn_node.append([int(j), 0])
                conn_k.append(k_leg); conn_rest.append(0.0)
    inp = _assemble("millipede_swarm", nodes_list, Q_list, dt, density=DENSITY, youngs=youngs,
                    radius=np.array(radius), damping=0.0, bc_start=0, bc_end=0)
    inp.conn_rod = np.array(conn_rod, np.int32)
    inp.conn_node = np.array(conn_node, np.int32)
    inp.conn_k = np.array(conn_k, float)
    inp.conn_c = np.full(len(conn_k), float(c_conn))
    inp.conn_rest = np.array(conn_rest, float)
    inp.magnetization = np.ascontiguousarray(np.concatenate(mag))
    inp.field = np.array([0.0, 0.0, 0.0, 0.0, 0.0, b0, b0, 0.0, 0.0])
    inp.field_freq = float(freq)
    return inp
