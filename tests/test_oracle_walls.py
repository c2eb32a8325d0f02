"""Pins of the oracle's planar walls (Results, "Active matter" and "Fibrous
granular materials": filaments confined by boundaries and in frictional
contact with them; the contact model is in the unavailable supplement, so the
reading is a penalty contact per node, a sphere of the rod's radius, with
damping proportional to the penetration and regularised Coulomb friction):

* a straight rod lying on the floor under gravity settles with every node
  sunk by its own weight over the stiffness, delta_j = m_j g / k;
* released sliding along the floor it decelerates at mu g (Coulomb) until the
  slip speed;
* dropped onto the floor without damping or friction it bounces with
  T + U + W_ext (gravity and the penalty potential) conserved to O(h^2);
* a rod out of contact feels nothing.  (A wall is a solid half-space n.x < d:
  rods live on the side of its normal.)
"""
import numpy as np

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC

N, L, RAD = 10, 0.1, 0.005
FLOOR = np.array([[0.0, 0.0, 1.0, 0.0]])


def _rod(z, k=100.0, c=0.0, mu=0.0, damping=0.0, vel=None, dt=1e-5, vslip=1e-4):
    nodes, Q = W.straight_rod(N, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(0.0, 0.0, z))
    inp = RC.single(nodes, Q, E=1e6, radius=RAD, damping=damping, dt=dt, vel=vel)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.walls = FLOOR.copy()
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = k, c, mu, vslip
    return inp


def _masses():
    A, _ = RC.section(RAD)
    m = np.full(N + 1, 1000.0 * A * L / N)
    m[0] = m[-1] = 0.5 * m[0]
    return m


def test_resting_rod_sinks_by_its_weight():
    """At rest the floor carries the whole weight: sum_j k delta_j = M g (the
    rod bends a little, since its end nodes carry half the load of the others);
    a one-element rod, whose two nodes carry equal loads, sinks uniformly by
    exactly m g / k."""
    k = 100.0
    o = ro.Oracle(_rod(RAD, k=k, c=500.0, damping=5.0))
    o.step(100000)
    M = _masses().sum()
    carried = k * np.sum(RAD - o.pos[:, 2])
    print("floor force", carried, "weight", M * 9.81)
    assert abs(carried / (M * 9.81) - 1) < 1e-8
    nodes, Q = W.straight_rod(1, 0.01, direction=(1, 0, 0), d1=(0, 1, 0), origin=(0.0, 0.0, RAD))
    one = RC.single(nodes, Q, E=1e6, radius=RAD, damping=5.0, dt=1e-5)
    one.gravity = np.array([0.0, 0.0, -9.81])
    one.walls = FLOOR.copy()
    one.wall_k, one.wall_c, one.wall_mu = k, 500.0, 0.0
    o1 = ro.Oracle(one)
    o1.step(100000)
    m = 0.5 * 1000.0 * np.pi * RAD ** 2 * 0.01
    assert np.abs(o1.pos[:, 2] - (RAD - m * 9.81 / k)).max() < 1e-10


def test_sliding_rod_decelerates_at_mu_g():
    k, mu, v0 = 100.0, 0.3, 0.5
    z0 = RAD - _masses() * 9.81 / k          # start at the resting penetration
    inp = _rod(RAD, k=k, c=500.0, mu=mu, vel=np.tile([v0, 0.0, 0.0], (N + 1, 1)))
    inp.position[:, 2] = z0
    o = ro.Oracle(inp)
    for _ in range(5):
        o.step(2000)
        vx = o.vel[:, 0].mean()
        want = v0 - mu * 9.81 * o.time
        print(o.time, vx, want)
        assert abs(vx - want) < 1e-3 * v0


def test_bounce_conserves_energy():
    o = ro.Oracle(_rod(0.02, k=200.0, dt=5e-6))
    H0 = o.energy().sum()
    H, zmin = [], 1.0
    for _ in range(40):
        o.step(2000)
        H.append(o.energy().sum())
        zmin = min(zmin, o.pos[:, 2].min())
    drift = np.abs(np.array(H) - H0).max() / abs(o.energy()[:, :4].sum() + 1e-30)
    print("lowest node", zmin, "energy drift / (T + U)", drift)
    assert zmin < RAD                        # it did hit the floor
    assert np.abs(np.array(H) - H0).max() < 1e-3 * 0.5 * 1000 * np.pi * RAD ** 2 * L * 9.81 * 0.02


def test_no_force_out_of_contact():
    """A rod held above the floor by more than its radius feels no wall: with no
    gravity it stays exactly where it is."""
    inp = _rod(0.05)
    inp.gravity = np.zeros(3)
    o = ro.Oracle(inp)
    o.step(100)
    assert np.array_equal(o.pos, inp.position)
