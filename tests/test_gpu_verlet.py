"""Verlet lists of rod-rod contact (node spheres and capsules, contact_skin).

Every node sums its contacts over its list in increasing node order, and a
pair missing from the lists cannot touch, so a run's results do not depend on
the skin or on when the lists were built: the tests compare runs with
different skins bit for bit, a resumed run with an uninterrupted one, runs
without lists and with overflowing lists (those nodes' contacts summed in
grid order) against the FP64 oracle, and at full size the lists against the
grid pass of every step.
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from test_gpu_step import _rod, assert_norms, run_both

pytestmark = pytest.mark.gpu


def _small_pile(seed=91):
    return W.fibre_pile(n_rods=24, n=20, L=0.2, per_row=2, rows=4, noise=1e-2, seed=seed)


def _bundle(r=0.01, n=24, seed=7):
    """Seven parallel rods along x in a hexagonal bundle (axes 2 r apart less
    1e-6 m, so neighbours touch), nodes one radius apart, no gravity, small
    random node velocities.  Within 2 r + 2 r of a node of the middle rod lie
    7 nodes of each of its 6 neighbours: 42 partners, more than a list holds."""
    rng = np.random.default_rng(seed)
    L = n * r
    d = 2.0 * r - 1e-6
    axes = [(0.0, 0.0)] + [(d * np.cos(a), d * np.sin(a)) for a in np.arange(6) * np.pi / 3]
    nodes, Qs, vel = [], [], []
    for (y, z) in axes:
        x, Q = W.straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0), origin=(0.0, y, z))
        nodes.append(x)
        Qs.append(Q)
        vel.append(rng.normal(0.0, 1e-2, size=(n + 1, 3)))
    inp = W._assemble("bundle", nodes, Qs, 1e-5, density=W.DENSITY, youngs=1e7, radius=r, damping=0.5,
                      bc_start=0, bc_end=0, velocity_list=vel)
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 1e5, 1e3, 0.3, 1e-2
    inp.rod_contact = 1
    return inp


def _run(inp, steps, precision="f64", **kw):
    R = _rod()
    with R.RodBatch(inp, precision=precision, **kw) as b:
        b.step(steps)
        out = b.get_state()[:4] + (b.energy(),)
        stats = b.contact_stats()
    return out, stats


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_skin_does_not_change_results():
    """A skin of 1e-9 m (a build almost every step), the default (a fifth of
    the radius) and two radii: the same bits after 1000 FP64 steps (energies
    included) and 400 FP32 steps; the smallest skin rebuilds far more often."""
    inp = _small_pile(seed=93)
    out = {}
    for skin in (1e-9, 0.0, 0.02):
        print(f"case: fibre pile 24 rods, FP64, 1000 steps, contact_skin={skin}", flush=True)
        out[skin] = _run(inp, 1000, contact_skin=skin)
        print("stats", out[skin][1], flush=True)
    for skin in (0.0, 0.02):
        assert _same(out[1e-9][0], out[skin][0]), skin
    tiny, dflt = out[1e-9][1], out[0.0][1]
    assert tiny["passes"] == dflt["passes"] == 1001   # 1000 steps and one energy call
    assert tiny["builds"] > 10 * dflt["builds"] and dflt["builds"] >= 1
    assert tiny["fallbacks"] == dflt["fallbacks"] == 0
    f32 = [_run(inp, 400, "f32", contact_skin=skin)[0] for skin in (1e-9, 0.0)]
    print("case: the same pile, FP32, 400 steps, two skins", flush=True)
    assert _same(*f32)


def test_resume_with_lists_is_bitwise():
    """300 steps, then 300 more, against a fresh batch given the state after
    300 (its lists built anew): the same bits."""
    R = _rod()
    inp = _small_pile(seed=97)
    print("case: fibre pile 24 rods, FP64, 600 steps against 300 + resume + 300", flush=True)
    with R.RodBatch(inp, precision="f64") as b:
        b.step(300)
        mid = b.get_state()
        b.step(300)
        whole = b.get_state()[:4]
    with R.RodBatch(inp, precision="f64") as b:
        b.set_state(*mid[:4], t=mid[4])
        b.step(300)
        resumed = b.get_state()[:4]
    assert _same(whole, resumed)


def test_no_lists_matches_oracle():
    print("case: fibre pile 24 rods, FP64, 1000 steps, contact_skin=-1 (no lists)", flush=True)
    norms, _ = run_both(_small_pile(seed=91), 1000, contact_skin=-1.0)
    assert_norms(norms)


def test_overflowing_lists_fall_back_to_grid_order():
    """With a skin of two radii the middle rod's nodes of the bundle have 42
    partners: every pass rebuilds, finds the overflow, sums those nodes'
    contacts in grid order and asks the next pass to build again; against the
    oracle as every contact test.  With the default skin (a fifth of the
    radius: 6 partners) the lists hold."""
    R = _rod()
    inp = _bundle()
    print("case: 7-rod bundle, FP64, 1000 steps, contact_skin=0.02 (overflowing lists)", flush=True)
    norms, _ = run_both(inp, 1000, contact_skin=0.02)
    assert_norms(norms)
    with R.RodBatch(inp, precision="f64", contact_skin=0.02) as b:
        b.step(50)
        s = b.contact_stats()
    print("stats", s, flush=True)
    assert s["passes"] == s["builds"] == s["fallbacks"] == 50 and s["most_partners"] > s["capacity"]
    print("case: 7-rod bundle, FP64, 1000 steps, default skin", flush=True)
    norms, _ = run_both(inp, 1000)
    assert_norms(norms)
    with R.RodBatch(inp, precision="f64") as b:
        b.step(50)
        s = b.contact_stats()
    print("stats", s, flush=True)
    assert s["fallbacks"] == 0 and 0 < s["most_partners"] <= s["capacity"]


def test_full_pile_lists_against_grid_pass():
    """16,384 fibres x 50 (835,584 nodes), 200 FP64 steps: a skin of 1e-6 m
    (a build every few steps) gives the default skin's bits; without lists
    the contacts are summed in grid order, so positions differ by rounding
    only (below 1e-12 m; one missed contact of the light initial overlaps
    would move a node by about 1e-10 m per step)."""
    inp = W.fibre_pile()
    runs = {}
    for skin in (1e-6, 0.0, -1.0):
        print(f"case: fibre pile 16384 x 50, FP64, 200 steps, contact_skin={skin}", flush=True)
        runs[skin] = _run(inp, 200, contact_skin=skin, tile_waves=4)
        print("stats", runs[skin][1], flush=True)
    assert _same(runs[1e-6][0], runs[0.0][0])
    assert runs[1e-6][1]["builds"] > 5 and runs[1e-6][1]["fallbacks"] == 0
    dpos = np.abs(runs[0.0][0][0] - runs[-1.0][0][0]).max()
    dvel = np.abs(runs[0.0][0][1] - runs[-1.0][0][1]).max()
    print(f"lists against grid pass: max |dpos| {dpos:.2e} m, max |dvel| {dvel:.2e} m/s", flush=True)
    assert dpos < 1e-12 and dvel < 1e-8


# ------------------------------------------------------------------ capsules
def _capsule_pile(seed=61):
    """Crossed layers of 2 x 4 fibres of 8 elements (3.1 radii each) on the
    floor in capsule contact, under gravity, with friction."""
    return W.fibre_pile(n_rods=24, n=8, L=0.248, per_row=2, rows=4, noise=1e-2, seed=seed, contact=2)


def test_capsule_skin_does_not_change_results():
    """Capsule lists: a skin of 1e-9 m, the default and two radii give the
    same bits after 1000 FP64 steps (energies included) and 400 FP32 steps;
    the smallest skin rebuilds far more often."""
    inp = _capsule_pile(seed=63)
    out = {}
    for skin in (1e-9, 0.0, 0.02):
        print(f"case: capsule pile 24 rods, FP64, 1000 steps, contact_skin={skin}", flush=True)
        out[skin] = _run(inp, 1000, contact_skin=skin)
        print("stats", out[skin][1], flush=True)
    for skin in (0.0, 0.02):
        assert _same(out[1e-9][0], out[skin][0]), skin
    tiny, dflt = out[1e-9][1], out[0.0][1]
    assert tiny["passes"] == dflt["passes"] == 1001
    assert tiny["builds"] > 10 * dflt["builds"] and dflt["builds"] >= 1
    assert tiny["fallbacks"] == dflt["fallbacks"] == 0 and dflt["most_partners"] > 0
    print("case: the same capsule pile, FP32, 400 steps, two skins", flush=True)
    f32 = [_run(inp, 400, "f32", contact_skin=skin)[0] for skin in (1e-9, 0.0)]
    assert _same(*f32)


def test_capsule_resume_with_lists_is_bitwise():
    R = _rod()
    inp = _capsule_pile(seed=67)
    print("case: capsule pile 24 rods, FP64, 600 steps against 300 + resume + 300", flush=True)
    with R.RodBatch(inp, precision="f64") as b:
        b.step(300)
        mid = b.get_state()
        b.step(300)
        whole = b.get_state()[:4]
    with R.RodBatch(inp, precision="f64") as b:
        b.set_state(*mid[:4], t=mid[4])
        b.step(300)
        resumed = b.get_state()[:4]
    assert _same(whole, resumed)


def test_capsule_no_lists_matches_oracle():
    print("case: capsule pile 24 rods, FP64, 1000 steps, contact_skin=-1 (no lists)", flush=True)
    norms, _ = run_both(_capsule_pile(seed=61), 1000, contact_skin=-1.0)
    assert_norms(norms)


def test_capsule_overflowing_lists_fall_back_to_grid_order():
    """The bundle's elements as capsules with a skin of four radii: more than
    32 elements within reach of the middle rod's elements, so every pass
    rebuilds and sums those elements' contacts in grid order; against the
    oracle, and with the default skin the lists hold."""
    R = _rod()
    inp = _bundle()
    inp.rod_contact = 2
    print("case: 7-rod bundle as capsules, FP64, 1000 steps, contact_skin=0.04 (overflowing lists)", flush=True)
    norms, _ = run_both(inp, 1000, contact_skin=0.04)
    assert_norms(norms)
    with R.RodBatch(inp, precision="f64", contact_skin=0.04) as b:
        b.step(50)
        s = b.contact_stats()
    print("stats", s, flush=True)
    assert s["passes"] == s["builds"] == s["fallbacks"] == 50 and s["most_partners"] > s["capacity"]
    print("case: 7-rod bundle as capsules, FP64, 1000 steps, default skin", flush=True)
    norms, _ = run_both(inp, 1000)
    assert_norms(norms)
    with R.RodBatch(inp, precision="f64") as b:
        b.step(50)
        s = b.contact_stats()
    print("stats", s, flush=True)
    assert s["fallbacks"] == 0 and 0 < s["most_partners"] <= s["capacity"]


def test_full_capsule_pile_lists_against_grid_pass():
    """16,384 fibres x 20 capsules, 200 FP64 steps: a skin of 1e-6 m gives
    the default skin's bits; the grid pass of every step sums in grid order,
    so positions differ by rounding only (below 1e-12 m)."""
    inp = W.capsule_pile()
    runs = {}
    for skin in (1e-6, 0.0, -1.0):
        print(f"case: capsule pile 16384 x 20, FP64, 200 steps, contact_skin={skin}", flush=True)
        runs[skin] = _run(inp, 200, contact_skin=skin, tile_waves=4)
        print("stats", runs[skin][1], flush=True)
    assert _same(runs[1e-6][0], runs[0.0][0])
    assert runs[1e-6][1]["builds"] > 5 and runs[1e-6][1]["fallbacks"] == 0
    dpos = np.abs(runs[0.0][0][0] - runs[-1.0][0][0]).max()
    dvel = np.abs(runs[0.0][0][1] - runs[-1.0][0][1]).max()
    print(f"lists against grid pass: max |dpos| {dpos:.2e} m, max |dvel| {dvel:.2e} m/s", flush=True)
    assert dpos < 1e-12 and dvel < 1e-8


@pytest.mark.parametrize("mode", [1, 2])
def test_lists_after_a_non_finite_rod(mode):
    """A node of rod 0 set to NaN: rod 0 is flagged (a non-finite node or
    element fails every distance test and is not binned, so contact carries
    no NaN; the step's exchange between neighbouring rods of a tile can, and
    those rods are flagged too).  With the state set back the lists are valid
    again (rebuilt where a build position went NaN), and the next 200 steps
    give the bits of a fresh batch given the same state."""
    R = _rod()
    inp = _small_pile(seed=101) if mode == 1 else _capsule_pile(seed=103)
    print(f"case: {'fibre' if mode == 1 else 'capsule'} pile 24 rods, FP64, NaN node in rod 0, then restored",
          flush=True)
    with R.RodBatch(inp, precision="f64") as b:
        b.step(100)
        pos, vel, dr, om, t = b.get_state()
        bad = pos.copy()
        bad[3] = np.nan   # a node of rod 0
        b.set_state(bad, vel, dr, om, t=t)
        b.step(50)
        flags = b.flags()
        assert flags[0] & R.ROD_FLAG_NONFINITE
        print("rods flagged", int((flags & R.ROD_FLAG_NONFINITE).astype(bool).sum()), "of", len(flags), flush=True)
        b.set_state(pos, vel, dr, om, t=t)
        assert not b.flags().any()
        b.step(200)
        after = b.get_state()[:4]
        print("stats", b.contact_stats(), flush=True)
    with R.RodBatch(inp, precision="f64") as c:
        c.set_state(pos, vel, dr, om, t=t)
        c.step(200)
        fresh = c.get_state()[:4]
    assert _same(after, fresh)
