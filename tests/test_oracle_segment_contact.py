"""Pins of the oracle's capsule (segment) contact, rod_contact = 2 (Results,
"Fibrous granular materials": filaments of high aspect ratio in frictional
contact; the contact law is in the unavailable supplement, so the reading is
the walls' law between the closest points of two elements' segments, each
element a capsule of its rod's radius, the force on an element shared by its
two nodes by the closest point's parameter; elements of one rod touch when the
rest lengths between them add up to at least the diameter):

* the closest-point routine against a dense grid search and a library
  minimiser on random segment pairs, and closed forms (perpendicular crossing,
  parallel offset, collinear gap);
* two rods whose elements are five radii long cross at right angles, the
  crossing in the middle of an element of each: with capsules they collide
  and part (momentum exact, T + U + W_ext conserved without damping or
  friction), while node spheres let them pass through each other;
* a rod folded into a hairpin with its arms closer than a diameter opens by
  self-contact (linear momentum exact, energy conserved), and a straight rod
  whose elements are shorter than its diameter steps bit for bit as without
  contact (the neighbours within a diameter are excluded);
* a short rod lying across a clamped rod under gravity settles on the single
  contact with k delta = M g.
"""
import numpy as np
import pytest

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W

RAD = 0.005


def _dist(p0, p1, q0, q1, s, t):
    return np.linalg.norm((p0 + s * (p1 - p0)) - (q0 + t * (q1 - q0)))


def test_segment_closest_points():
    from scipy.optimize import minimize
    rng = np.random.default_rng(4)
    grid = np.linspace(0.0, 1.0, 201)
    S, T = np.meshgrid(grid, grid, indexing="ij")
    for k in range(60):
        p0, p1, q0, q1 = rng.normal(size=(4, 3))
        if k % 10 == 0:          # parallel pairs
            q1 = q0 + 0.7 * (p1 - p0)
        if k % 10 == 1:          # a shared end point
            q0 = p1.copy()
        s, t = ro.segment_closest(p0, p1, q0, q1)
        assert 0.0 <= s <= 1.0 and 0.0 <= t <= 1.0
        d = _dist(p0, p1, q0, q1, s, t)
        P = p0[None, None, :] + S[..., None] * (p1 - p0)
        Q = q0[None, None, :] + T[..., None] * (q1 - q0)
        assert d <= np.linalg.norm(P - Q, axis=2).min() + 1e-12
        res = minimize(lambda x: _dist(p0, p1, q0, q1, x[0], x[1]) ** 2, x0=[0.5, 0.5],
                       bounds=[(0, 1), (0, 1)], method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12})
        assert d <= np.sqrt(res.fun) + 1e-7
    z = np.zeros(3)
    ex, ey, ez = np.eye(3)
    assert ro.segment_closest(-ex, ex, -ey + ez, ey + ez) == (0.5, 0.5)
    s, t = ro.segment_closest(z, ex, ey, ex + ey)             # parallel, offset 1
    assert abs(_dist(z, ex, ey, ex + ey, s, t) - 1.0) < 1e-15
    assert ro.segment_closest(z, ex, 2 * ex, 3 * ex) == (1.0, 0.0)   # collinear, gap 1


def test_segment_distance_moves_no_more_than_the_end_points():
    """The property capsule Verlet lists rest on: when each end point of two
    segments moves by at most e, every point of either moves by at most e (a
    convex combination), so their closest distance changes by at most 2 e.
    Random pairs (near-parallel and end-sharing ones included) and random
    moves of every end point, the distances from the oracle's routine."""
    rng = np.random.default_rng(12)
    worst = 0.0
    for k in range(400):
        p0, p1, q0, q1 = rng.normal(size=(4, 3))
        if k % 8 == 0:
            q1 = q0 + 0.7 * (p1 - p0) + 1e-7 * rng.normal(size=3)   # near-parallel
        if k % 8 == 1:
            q0 = p1.copy()
        d = _dist(p0, p1, q0, q1, *ro.segment_closest(p0, p1, q0, q1))
        e = 10.0 ** rng.uniform(-6, -1)
        mv = rng.normal(size=(4, 3))
        mv *= (e * rng.uniform(0.0, 1.0, size=(4, 1))) / np.linalg.norm(mv, axis=1, keepdims=True)
        a0, a1, b0, b1 = p0 + mv[0], p1 + mv[1], q0 + mv[2], q1 + mv[3]
        d2 = _dist(a0, a1, b0, b1, *ro.segment_closest(a0, a1, b0, b1))
        assert abs(d2 - d) <= 2 * e + 1e-12, (k, d, d2, e)
        worst = max(worst, abs(d2 - d) / (2 * e))
    assert worst > 0.5   # the bound is approached, so the test can see a violation


def _long_crossing(mode, gap=2e-4, vz=-0.5, n=4, L=0.1):
    """Rod A along x and rod B along y (above A by 2 RAD + gap, moving with
    vz), elements L / n = 5 RAD long, the crossing at the middle of element 1 of
    each (nodes at -3 l/2, -l/2, l/2, 3 l/2, 5 l/2)."""
    lh = L / n
    a_nodes, a_Q = W.straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(-1.5 * lh, 0.0, 0.0))
    b_nodes, b_Q = W.straight_rod(n, L, direction=(0, 1, 0), d1=(0, 0, 1), origin=(0.0, -1.5 * lh, 2 * RAD + gap))
    vel = [np.zeros((n + 1, 3)), np.tile([0.0, 0.0, vz], (n + 1, 1))]
    inp = W._assemble("long crossing", [a_nodes, b_nodes], [a_Q, b_Q], 1e-5, density=1000.0, youngs=1e6,
                      radius=RAD, damping=0.0, bc_start=0, bc_end=0, velocity_list=vel)
    inp.rod_contact = mode
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 100.0, 0.0, 0.0, 1e-4
    return inp


def _mass_vec(inp):
    A = np.pi * inp.radius ** 2
    out = []
    for r, n in enumerate(inp.n_elems):
        x = inp.position[inp.node_offset[r]:inp.node_offset[r] + n + 1]
        lh = np.linalg.norm(np.diff(x, axis=0), axis=1)
        m = np.zeros(n + 1)
        m[:-1] += 0.5 * inp.density[r] * A[r] * lh
        m[1:] += 0.5 * inp.density[r] * A[r] * lh
        out.append(m)
    return np.concatenate(out)


def test_long_elements_collide_as_capsules_and_pass_as_spheres():
    caps = _long_crossing(2)
    o = ro.Oracle(caps)
    m = _mass_vec(caps)
    p0 = (m[:, None] * o.vel).sum(0)
    H0 = o.energy().sum()
    na = caps.n_elems[0] + 1

    def rel(ob):   # B's mean height and vertical velocity relative to A's
        return (ob.pos[na:, 2].mean() - ob.pos[:na, 2].mean(), ob.vel[na:, 2].mean() - ob.vel[:na, 2].mean())

    zmin, H = 1.0, []
    for _ in range(60):
        o.step(100)
        zmin = min(zmin, rel(o)[0])
        H.append(o.energy().sum())
    p1 = (m[:, None] * o.vel).sum(0)
    assert np.abs(p1 - p0).max() <= 1e-12 * np.abs(p0).max()
    z1, w1 = rel(o)
    print("capsules: closest approach", zmin / RAD, "radii; final separation speed", w1)
    assert w1 > 0.0                             # the rods move apart again
    assert zmin > RAD                           # B's axis never came within one radius of A's
    assert max(abs(h - H0) for h in H) <= 1e-3 * H0
    spheres = _long_crossing(1)
    o1 = ro.Oracle(spheres)
    o1.step(6000)
    print("spheres: final separation", rel(o1)[0] / RAD, "radii")
    assert rel(o1)[0] < -2 * RAD                # node spheres: B passed through A


def _hairpin(gap, n_arm=12, lh=0.01, rad=RAD):
    """A rod bent into a hairpin: an arm along +x at y = 0, a semicircular
    turn of radius (2 rad + gap) / 2 made of straight elements, and an arm back
    along -x at y = 2 rad + gap (the arms' capsules gap apart)."""
    h = 2 * rad + gap
    pts = [np.array([-(n_arm * lh), 0.0, 0.0]) + np.array([k * lh, 0.0, 0.0]) for k in range(n_arm + 1)]
    n_turn = 6
    for k in range(1, n_turn + 1):
        a = -np.pi / 2 + np.pi * k / n_turn
        pts.append(np.array([0.5 * h * np.cos(a), 0.5 * h + 0.5 * h * np.sin(a), 0.0]))
    for k in range(1, n_arm + 1):
        pts.append(np.array([-k * lh, h, 0.0]))
    nodes = np.array(pts)
    return nodes


def test_hairpin_opens_by_self_contact():
    from rodcases import single
    nodes = _hairpin(gap=-4e-4)
    Q = W.frames_parallel_transport(nodes, d1_first=(0.0, 0.0, 1.0))
    inp = single(nodes, Q, E=1e5, radius=RAD, rest_length=np.linalg.norm(np.diff(nodes, axis=0), axis=1))
    inp.rest_kappa = ro.Oracle(inp).strains()[1].copy()   # the hairpin is the rest shape
    inp.rod_contact = 2
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 20.0, 0.0, 0.0, 1e-4
    o = ro.Oracle(inp)
    m = _mass_vec(inp)
    H0 = o.energy().sum()
    assert o.energy()[0, 4] > 0.0               # the arms overlap: a contact potential
    n = inp.n_elems[0]
    arm_a, arm_b = slice(0, 12), slice(n - 11, n + 1)
    gap0 = o.pos[arm_b, 1].mean() - o.pos[arm_a, 1].mean()
    for _ in range(10):
        o.step(100)
        assert abs(o.energy().sum() - H0) <= 1e-3 * H0
    p = (m[:, None] * o.vel).sum(0)
    assert np.abs(p).max() <= 1e-12 * (m.sum() * np.abs(o.vel).max())
    gap1 = o.pos[arm_b, 1].mean() - o.pos[arm_a, 1].mean()
    assert gap1 > gap0                          # the arms were pushed apart
    # the same hairpin without contact: the arms do not move apart by themselves
    inp0 = inp.copy()
    inp0.rod_contact = 0
    o0 = ro.Oracle(inp0)
    o0.step(1000)
    assert o0.pos[arm_b, 1].mean() - o0.pos[arm_a, 1].mean() < gap1


def test_straight_rod_has_no_self_contact():
    """Elements 0.35 of a diameter long: elements with fewer than three
    elements between them overlap as capsules in the straight state and are
    excluded, the next ones are half a millimetre apart; the rod steps bit for
    bit as without contact."""
    from rodcases import single
    nodes, Q = W.straight_rod(20, 0.07, direction=(1, 0, 0), d1=(0, 1, 0))
    rng = np.random.default_rng(6)
    vel = rng.normal(scale=1e-3, size=nodes.shape)
    inp = single(nodes, Q, radius=RAD, vel=vel)
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 20.0, 1.0, 0.3, 1e-4
    a, b = inp.copy(), inp.copy()
    a.rod_contact, b.rod_contact = 2, 0
    oa, ob = ro.Oracle(a), ro.Oracle(b)
    oa.step(300)
    ob.step(300)
    for x, y in zip(oa.state(), ob.state()):
        assert np.array_equal(x, y)
    assert oa.energy()[0, 4] == 0.0


def test_rod_resting_across_a_clamped_rod():
    """A 3-element rod (elements 5 radii long) laid across the middle of a
    3-element rod clamped at both ends, the crossing in the middle of an
    element of each, under gravity with damping: it settles with its weight on
    the one contact, k delta = M g to 1e-4."""
    from rodcases import single  # noqa: F401
    n, L = 3, 0.075
    lh = L / n
    lower, lQ = W.straight_rod(3, 0.03, direction=(1, 0, 0), d1=(0, 1, 0), origin=(-0.015, 0.0, 0.0))
    upper, uQ = W.straight_rod(n, L, direction=(0, 1, 0), d1=(0, 0, 1), origin=(0.0, -1.5 * lh, 2 * RAD + 1e-4))
    inp = W._assemble("resting", [lower, upper], [lQ, uQ], 1e-5, density=1000.0, youngs=1e7, radius=RAD,
                      damping=50.0, bc_start=0, bc_end=0)
    inp.bc_start = np.array([1, 0], np.int32)
    inp.bc_end = np.array([1, 0], np.int32)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.rod_contact = 2
    k = 200.0
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = k, 0.0, 0.0, 1e-4
    o = ro.Oracle(inp)
    o.step(40000)
    M = 1000.0 * np.pi * RAD ** 2 * L
    low, up = o.pos[:4], o.pos[4:]
    s, t = ro.segment_closest(low[1], low[2], up[1], up[2])
    d = np.linalg.norm((low[1] + s * (low[2] - low[1])) - (up[1] + t * (up[2] - up[1])))
    delta = 2 * RAD - d
    print("k delta / M g", k * delta / (M * 9.81), "s, t", s, t)
    assert abs(k * delta / (M * 9.81) - 1.0) < 1e-4
    assert np.abs(o.vel[4:]).max() < 1e-5
