"""Pins of the oracle's rod-rod contact (Results, "Fibrous granular materials",
and the collision engine named as future work; the contact law is in the
unavailable supplement, so the reading is the walls' law between nodes of
different rods: each node a sphere of its rod's radius, overlap
delta = r_a + r_b - |x_a - x_b|, normal force delta (k - c v_n) along
x_a - x_b while positive, regularised Coulomb friction, potential 1/2 k delta^2
split between the two rods):

* two free rods crossing at right angles collide head-on without damping or
  friction: linear momentum exact (the pair's forces are equal and opposite),
  angular momentum (orbital + spin) and T + U + W_ext conserved, and the rods
  part again;
* the same collision with friction and a sideways approach: momentum still
  exact, energy lost (a friction force of the wrong sign would feed it);
* a rod laid on another on the floor settles into the grooves between the
  lower rod's nodes, its weight carried by the node contacts (the vertical
  components of k delta sum to M g), and the floor carries both rods;
* normal damping c takes energy out of a frictionless collision, more for a
  larger c, none for c = 0;
* a rod pressed by an end force F against the end of a clamped rod settles
  with the two touching nodes 2 r - F / k apart;
* contact off: far-apart rods, and a rod curled onto itself (no self-contact),
  step exactly as without contact.
"""
import numpy as np

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC

N, L, RAD = 10, 0.1, 0.005
FLOOR = np.array([[0.0, 0.0, 1.0, 0.0]])


def _crossing(gap, vel_b, k=10.0, c=0.0, mu=0.0, damping=0.0):
    """Rod A along x centred at the origin, rod B along y centred above it at
    height 2 RAD + gap, moving with vel_b: node 5 of each at the crossing."""
    a_nodes, a_Q = W.straight_rod(N, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(-L / 2, 0.0, 0.0))
    b_nodes, b_Q = W.straight_rod(N, L, direction=(0, 1, 0), d1=(0, 0, 1),
                                  origin=(0.0, -L / 2, 2 * RAD + gap))
    vel = [np.zeros((N + 1, 3)), np.tile(np.asarray(vel_b, float), (N + 1, 1))]
    inp = W._assemble("crossing", [a_nodes, b_nodes], [a_Q, b_Q], 1e-5, density=1000.0, youngs=1e6,
                      radius=RAD, damping=damping, bc_start=0, bc_end=0, velocity_list=vel)
    inp.rod_contact = 1
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = k, c, mu, 1e-4
    return inp


def _masses(inp):
    A = np.pi * inp.radius ** 2
    out = []
    for r, n in enumerate(inp.n_elems):
        lh = np.linalg.norm(np.diff(inp.position[inp.node_offset[r]:inp.node_offset[r] + n + 1], axis=0), axis=1)
        m = np.zeros(n + 1)
        m[:-1] += 0.5 * inp.density[r] * A[r] * lh
        m[1:] += 0.5 * inp.density[r] * A[r] * lh
        out.append(m)
    return np.concatenate(out)


def _momenta(o, m):
    p = (m[:, None] * o.vel).sum(0)
    Lo = np.cross(o.pos, m[:, None] * o.vel).sum(0)
    _, I = RC.section(RAD)
    J = 1000.0 * I * (L / N) * np.array([1.0, 1.0, 2.0])
    _, _, e = o.strains()
    spin = np.einsum("iba,ib->ia", o.dir, J * o.omega / e[:, None]).sum(0)
    return p, Lo + spin


def test_frictionless_collision_conserves_momenta_and_energy():
    inp = _crossing(gap=2e-4, vel_b=[0.0, 0.0, -0.05])
    o = ro.Oracle(inp)
    m = _masses(inp)
    p0, L0 = _momenta(o, m)
    H0 = o.energy().sum()
    H, closest = [], 1.0
    for _ in range(40):
        o.step(100)
        H.append(o.energy().sum())
        closest = min(closest, o.pos[11 + 5, 2] - o.pos[5, 2])
    p1, L1 = _momenta(o, m)
    drift = np.abs(np.array(H) - H0).max() / H0
    vz_rel = o.vel[11:, 2].mean() - o.vel[:11, 2].mean()
    print("closest approach", closest, "energy drift", drift, "relative vz after", vz_rel, "p", p0, p1)
    assert closest < 2 * RAD                   # the spheres overlapped
    assert vz_rel > 0                          # and the rods parted again
    assert np.abs(p1 - p0).max() < 1e-15
    assert np.abs(L1 - L0).max() < 1e-6 * np.abs(p0).max() * L
    # a potential of the wrong weight or a force of the wrong sign is O(1)
    assert drift < 1e-3


def test_friction_keeps_momentum_and_dissipates():
    out = {}
    for mu in (0.0, 0.5):
        inp = _crossing(gap=2e-4, vel_b=[0.03, 0.0, -0.05], mu=mu)
        o = ro.Oracle(inp)
        m = _masses(inp)
        p0, _ = _momenta(o, m)
        H0 = o.energy().sum()
        o.step(4000)
        p1, _ = _momenta(o, m)
        assert np.abs(p1 - p0).max() < 1e-15
        out[mu] = (o.energy().sum() - H0) / H0
        # relative sliding velocity (x) of the upper rod's crossing node
        out[(mu, "slide")] = o.vel[11 + 5, 0] - o.vel[5, 0]
    print(out)
    assert abs(out[0.0]) < 1e-3
    assert out[0.5] < -1e-3                    # friction took energy out
    assert out[(0.5, "slide")] < out[(0.0, "slide")]   # and slowed the sliding


def test_stacked_rods_carry_the_upper_weight():
    k = 50.0
    lo_nodes, lo_Q = W.straight_rod(N, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(0.0, 0.0, RAD))
    # the upper rod starts half an element along, over the grooves between the
    # lower rod's nodes, where it settles (stacked node on node is unstable)
    hi_nodes, hi_Q = W.straight_rod(N, L, direction=(1, 0, 0), d1=(0, 1, 0),
                                    origin=(0.5 * L / N, 0.0, 3 * RAD))
    inp = W._assemble("stack", [lo_nodes, hi_nodes], [lo_Q, hi_Q], 1e-5, density=1000.0, youngs=1e6,
                      radius=RAD, damping=10.0, bc_start=0, bc_end=0)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.walls = FLOOR.copy()
    inp.rod_contact = 1
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = k, 500.0, 0.0, 1e-4
    o = ro.Oracle(inp)
    o.step(200000)
    m = _masses(inp)
    M_lo, M_hi = m[:N + 1].sum(), m[N + 1:].sum()
    # vertical support of the upper rod: every overlapping node pair's normal
    # force k delta, times the normal's z component (the upper rod settles
    # into the grooves between the lower rod's nodes)
    d = o.pos[N + 1:, None, :] - o.pos[None, :N + 1, :]
    dist = np.linalg.norm(d, axis=2)
    delta = np.clip(2 * RAD - dist, 0.0, None)
    carried = k * np.sum(delta * d[:, :, 2] / dist)
    floor = k * np.sum(np.clip(RAD - o.pos[:N + 1, 2], 0.0, None))
    print("upper", carried / (M_hi * 9.81), "floor", floor / ((M_lo + M_hi) * 9.81),
          "shift", o.pos[N + 1, 0] - o.pos[0, 0])
    # at rest to 1e-6 (the damped settling is exponential); a force of the
    # wrong law or weight is off by O(1)
    assert abs(carried / (M_hi * 9.81) - 1) < 1e-6
    assert abs(floor / ((M_lo + M_hi) * 9.81) - 1) < 1e-6


def test_no_contact_changes_nothing():
    # far apart
    inp = _crossing(gap=0.05, vel_b=[0.0, 0.0, -0.01])
    off = inp.copy()
    off.rod_contact = 0
    a, b = ro.Oracle(inp), ro.Oracle(off)
    a.step(300)
    b.step(300)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)
    # one rod curled so that its own nodes overlap: a rod does not touch itself
    nodes, Q = RC.polygon_arc(12, 0.005, 2 * np.pi / 11)
    one = RC.single(nodes, Q, radius=RAD, dt=1e-5, vel=np.tile([0.0, 0.0, 0.01], (13, 1)))
    one.rod_contact = 1
    one.wall_k, one.wall_c = 10.0, 0.0
    assert np.linalg.norm(nodes[0] - nodes[10]) < 2 * RAD     # it does overlap itself
    two = one.copy()
    two.rod_contact = 0
    a, b = ro.Oracle(one), ro.Oracle(two)
    a.step(300)
    b.step(300)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.vel, b.vel)


def test_contact_damping_dissipates_in_proportion():
    """Head-on frictionless collisions with growing normal damping c: the energy
    after the collision falls as c grows (the damping term delta c v_n opposes
    the approach and the separation), and with c = 0 it is conserved; a damping
    of the wrong sign would feed energy."""
    lost = []
    for c in (0.0, 1.0, 4.0):
        inp = _crossing(gap=2e-4, vel_b=[0.0, 0.0, -0.05], c=c)
        o = ro.Oracle(inp)
        H0 = o.energy().sum()
        o.step(4000)
        lost.append((H0 - o.energy().sum()) / H0)
    print("relative energy lost", lost)
    assert abs(lost[0]) < 1e-3
    assert 0 < lost[1] < lost[2]


def _press(k, F, na=5, nb=5):
    """Rod A (clamped at both ends) and rod B on the x axis, B's first node
    touching A's last; an end force -F x on B's last node."""
    a_nodes, a_Q = W.straight_rod(na, 0.05, direction=(1, 0, 0), d1=(0, 1, 0), origin=(-0.05, 0.0, 0.0))
    b_nodes, b_Q = W.straight_rod(nb, 0.05, direction=(1, 0, 0), d1=(0, 1, 0), origin=(2 * RAD, 0.0, 0.0))
    inp = W._assemble("press", [a_nodes, b_nodes], [a_Q, b_Q], 1e-5, density=1000.0, youngs=1e6, radius=RAD,
                      damping=np.array([0.0, 30.0]), bc_start=np.array([1, 0]), bc_end=np.array([1, 0]),
                      end_force=np.array([[0.0, 0.0, 0.0], [-F, 0.0, 0.0]]))
    inp.rod_contact = 1
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = k, 0.0, 0.0, 1e-4
    return inp


def test_static_load_on_a_clamped_rod():
    """A clamped rod A and a free rod B on one line along x, B's first node
    touching A's last; an end force F on B's last node presses B against A.
    With damping B settles where the contact carries F: the two nodes sit
    2 r - F / k apart (Hooke's law of the penalty), independent of B's own
    compression."""
    k, F = 40.0, 2e-3
    na = 5
    inp = _press(k, F)
    o = ro.Oracle(inp)
    o.step(100000)
    gap = o.pos[na + 1, 0] - o.pos[na, 0]
    print("gap", gap, "want", 2 * RAD - F / k, "residual speed", np.abs(o.vel).max())
    assert abs(gap - (2 * RAD - F / k)) < 1e-8
