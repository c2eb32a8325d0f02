"""GPU parity of rod-rod contact (nodes as spheres of the rod radius, the
walls' penalty law between nodes of different rods, pairs found by the
hashed grid) against the FP64 oracle's brute force over all node pairs,
through the C boundary.  Bars on all five norms as in test_gpu_step (FP64: 3 x
the oracle's one-ulp conditioning; FP32: 4 x its FP32 mirror's discrepancy),
energies (W_ext holding the contact potentials) included.
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from test_gpu_step import _rod, assert_norms, run_both
import test_oracle_contact as OC

pytestmark = pytest.mark.gpu


def _small_pile(seed=91):
    """Three crossed layers of 8 fibres of 20 elements (1 cm elements, radius
    1 cm) on the floor, under gravity, with friction."""
    return W.fibre_pile(n_rods=24, n=20, L=0.2, per_row=2, rows=4, noise=1e-2, seed=seed)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_fibre_pile_f64(waves):
    print(f"case: fibre pile 24 rods x 20, tile_waves={waves}, FP64, 1000 steps", flush=True)
    norms, info = run_both(_small_pile(), 1000, tile_waves=waves)
    assert info["tile_waves"] == waves and info["substeps"] == 1
    assert_norms(norms)


def test_crossing_collision_f64():
    print("case: two crossing rods colliding with friction, FP64, 4000 steps", flush=True)
    inp = OC._crossing(gap=2e-4, vel_b=[0.03, 0.0, -0.05], mu=0.5, c=2.0)
    norms, _ = run_both(inp, 4000)
    assert_norms(norms)


def _linked_pile(seed=93):
    inp = _small_pile(seed=seed)
    pairs = [(2 * k, 2 * k + 1) for k in range(12)]
    inp.conn_rod = np.array(pairs, np.int32)
    inp.conn_node = np.array([[20, 0]] * len(pairs), np.int32)
    inp.conn_k = np.full(len(pairs), 50.0)
    inp.conn_c = np.full(len(pairs), 0.01)
    inp.conn_rest = np.array([np.linalg.norm(inp.position[inp.node_offset[b]] - inp.position[inp.node_offset[a] + 20])
                              for a, b in pairs])
    return inp


def test_pile_with_connections_f64():
    """Contact together with connections and walls: pairs of fibres joined
    end to end by springs."""
    print("case: fibre pile with end-to-end springs, FP64, 1000 steps", flush=True)
    norms, _ = run_both(_linked_pile(), 1000)
    assert_norms(norms)


def test_full_pile_conserves_momentum():
    """The full 16,384-fibre pile without gravity, floor, damping or friction:
    the contact forces come in equal and opposite pairs, so the total linear
    momentum stays at its initial value to round-off, and T + U + W_ext (the
    contact potentials summed by the grid pass) is conserved; the autotuned
    launch shape runs one step per launch."""
    print("case: fibre pile 16384 x 50, no gravity/floor/damping/friction, FP64, 200 steps", flush=True)
    R = _rod()
    inp = W.fibre_pile(overlap=2e-4, damping=0.0, mu=0.0, contact_c=0.0)
    inp.gravity = np.zeros(3)
    inp.walls = None
    A = np.pi * inp.radius ** 2
    m = np.zeros(inp.position.shape[0])
    for r, n in enumerate(inp.n_elems):
        o = inp.node_offset[r]
        m[o:o + n] += 0.5 * inp.density[r] * A[r] * (0.5 / n)
        m[o + 1:o + n + 1] += 0.5 * inp.density[r] * A[r] * (0.5 / n)
    p0 = (m[:, None] * inp.velocity).sum(0)
    with R.RodBatch(inp, precision="f64", autotune=True) as b:
        info = b.info()
        H0 = b.energy().sum()
        b.step(200)
        pos, vel, _, _, _ = b.get_state()
        e = b.energy()
    H1 = e.sum()
    print("energy", H0, H1, "relative drift", (H1 - H0) / H0, flush=True)
    p1 = (m[:, None] * vel).sum(0)
    scale = np.abs(m[:, None] * vel).sum()
    moved = np.abs(vel - inp.velocity).max()
    print("substeps", info["substeps"], "p0", p0, "p1", p1, "scale", scale, "max dv", moved, flush=True)
    assert info["substeps"] == 1
    assert np.isfinite(pos).all() and np.isfinite(e).all()
    assert moved > 1e-3                      # the initial overlaps pushed the layers apart
    assert np.abs(p1 - p0).max() < 1e-12 * scale
    # no damping, friction or dashpot: T + U + W_ext (contact potentials from the grid pass) holds
    assert abs(H1 - H0) < 1e-3 * abs(H0)       # measured 4.9e-5


def test_wrapped_grid_f64():
    """Two colliding pairs of crossing rods 20 m apart: the grid's cells per
    axis are capped by the bucket budget (4 per node), so the grid wraps many
    times over the batch's extent and far-apart nodes share buckets; the result
    must still be the oracle's."""
    print("case: two crossing pairs 20 m apart (wrapped grid), FP64, 3000 steps", flush=True)
    a = OC._crossing(gap=2e-4, vel_b=[0.0, 0.0, -0.05], mu=0.3, c=1.0)
    b = OC._crossing(gap=1e-4, vel_b=[0.02, 0.0, -0.04], mu=0.3, c=1.0)
    inp = a.copy()
    for f in ("n_elems", "velocity", "director", "omega", "density", "youngs", "shear_modulus", "radius",
              "shear_coeff", "damping", "bc_start", "bc_end"):
        setattr(inp, f, np.concatenate([getattr(a, f), getattr(b, f)]))
    inp.position = np.concatenate([a.position, b.position + np.array([20.0, 3.0, -1.0])])
    norms, _ = run_both(inp, 3000)
    assert_norms(norms)


def test_contact_graph_replays():
    """rod_step(100) five times (each a replay of the captured 64-step graph
    and of the 36-step graph of the rest, with eager work and synchronisations
    between the calls) against the oracle's 500 steps: every contact pass
    clears its bucket counts for the next, so replays after the first see a
    clean grid."""
    print("case: fibre pile 24 rods, 5 x rod_step(100) by captured graphs, FP64", flush=True)
    import torch
    R = _rod()
    inp = _small_pile(seed=95)
    from parity import oracle_pair, rod_norms, energy_norm, fp64_bars
    o, p = oracle_pair(inp, 500)
    with R.RodBatch(inp, precision="f64") as b:
        for k in range(5):
            b.step(100)
            torch.cuda.synchronize()
            _ = torch.ones(1024, device="cuda").sum().item()   # eager work between replays
        pos, vel, dr, om, t = b.get_state()
        e_gpu = b.energy()
    norms = rod_norms(inp, o.state(), (pos, vel, dr, om), 500 * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_gpu)
    norms["bars"], _ = fp64_bars(inp, o, p, 500)
    print("norms", {k: f"{v:.2e}" for k, v in norms.items() if k != "bars"}, flush=True)
    assert_norms(norms)


def test_contact_f32_parity():
    """FP32 batches: node positions for the grid summed along each rod in FP64
    from the FP32 edges; all five norms within the FP32 bars (4 x the FP32
    mirror's discrepancy from the FP64 oracle)."""
    cases = (("fibre pile 24 rods", _small_pile(seed=97), 1000),
             ("fibre pile with end-to-end springs", _linked_pile(seed=98), 1000),
             ("crossing collision with friction", OC._crossing(gap=2e-4, vel_b=[0.03, 0.0, -0.05], mu=0.5, c=2.0), 2000))
    for name, inp, steps in cases:
        print(f"case: {name}, FP32, {steps} steps", flush=True)
        norms, info = run_both(inp, steps, precision="f32")
        assert info["substeps"] == 1
        assert_norms(norms)


def _edge_case_input(mode=1):
    """Contact with everything else at once: rods of 1 to 100 elements and of
    different radii (the grid's cells follow the largest), some clamped at
    their base (a clamped node keeps its place whatever presses on it),
    magnetized elements in a rotating field, muscle moments, gravity and a
    floor; rods cross one above the other so that many pairs touch."""
    rng = np.random.default_rng(99)
    lengths = [1, 2, 3, 20, 63, 64, 65, 100, 5, 40]
    nodes_list, Q_list = [], []
    for k, n in enumerate(lengths):
        ds = 0.004
        direction = (1, 0, 0) if k % 2 == 0 else (0, 1, 0)
        d1 = (0, 1, 0) if k % 2 == 0 else (0, 0, 1)
        # every rod centred over (0.02, 0.02), alternately along x and y, 5 mm above the previous
        L = n * ds
        origin = (0.02 - L / 2, 0.02, 0.004 + 0.005 * k) if k % 2 == 0 else (0.02, 0.02 - L / 2, 0.004 + 0.005 * k)
        nodes, Q = W.straight_rod(n, n * ds, direction=direction, d1=d1, origin=origin)
        nodes_list.append(nodes)
        Q_list.append(Q)
    R = len(lengths)
    radii = rng.uniform(0.002, 0.004, R)
    vel = [rng.normal(0, 0.02, (n + 1, 3)) for n in lengths]
    inp = W._assemble("contact_edges", nodes_list, Q_list, 2e-6, density=1000.0, youngs=1e6, radius=radii,
                      damping=0.2, bc_start=np.array([k % 4 == 1 for k in range(R)], np.int32), bc_end=0,
                      velocity_list=vel)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.walls = np.array([[0.0, 0.0, 1.0, 0.0]])
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 20.0, 10.0, 0.3, 0.02
    inp.rod_contact = mode
    ne = int(np.sum(lengths))
    inp.magnetization = np.tile([0.0, 0.0, 1e-4], (ne, 1))
    inp.field = np.array([0.0, 0.0, 0.0, 0.01, 0.0, 0.0, 0.0, 0.01, 0.0])
    inp.field_freq = 5.0
    nv = ne - R
    inp.muscle_amp = np.full(nv, 1e-7)
    inp.muscle_axis = np.tile([1.0, 0.0, 0.0], (R, 1))
    inp.muscle_freq = np.full(R, 2.0)
    inp.muscle_wavenumber = np.full(R, 10.0)
    inp.muscle_phase = rng.uniform(0, 2 * np.pi, R)
    return inp


def test_contact_edge_cases_f64():
    print("case: contact edge cases (lengths 1..100, radii, clamps, field, muscles, floor), FP64, 1000 steps",
          flush=True)
    inp = _edge_case_input()
    from oracle import rodoracle as ro
    o = ro.Oracle(inp)
    d = o.pos[:, None, :] - o.pos[None, :, :]
    rod = np.repeat(np.arange(inp.n_rods), np.asarray(inp.n_elems) + 1)
    rr = inp.radius[rod]
    touching = (np.linalg.norm(d, axis=2) < rr[:, None] + rr[None, :]) & (rod[:, None] != rod[None, :])
    print("pairs in contact at the start", int(touching.sum()) // 2, flush=True)
    assert touching.sum() > 0
    norms, _ = run_both(inp, 1000)
    assert_norms(norms)


def test_press_against_clamped_rod_f64():
    """A rod pushed by an end force against a rod clamped at both ends (the
    oracle's static-load pin), 2000 steps of the approach to rest."""
    print("case: rod pressed against a clamped rod, FP64, 2000 steps", flush=True)
    norms, _ = run_both(OC._press(40.0, 2e-3), 2000)
    assert_norms(norms)


def test_contact_is_bitwise_repeatable_and_tile_invariant():
    """Each grid bucket is sorted by node id before the forces are summed, so
    a contact run gives the same bits every time and at every tile width (the
    contact pass does not depend on the tiles; the step kernel's arithmetic is
    the same at every width).  Two runs at 4-wave tiles and one at each other
    width of a 24-fibre pile, 500 FP64 steps, and two 300-step FP32 runs."""
    R = _rod()
    inp = _small_pile(seed=99)
    out = {}
    for tag, waves in (("a", 4), ("b", 4), ("w1", 1), ("w2", 2), ("w8", 8)):
        print(f"case: fibre pile 24 rods, FP64, tile_waves={waves}, run {tag}", flush=True)
        with R.RodBatch(inp, precision="f64", tile_waves=waves, substeps=1) as b:
            b.step(500)
            out[tag] = b.get_state()[:4] + (b.energy(),)
    for tag in ("b", "w1", "w2", "w8"):
        assert all(np.array_equal(x, y) for x, y in zip(out["a"], out[tag])), tag
    f32 = []
    for run in range(2):
        print(f"case: fibre pile 24 rods, FP32, run {run}", flush=True)
        with R.RodBatch(inp, precision="f32", tile_waves=2, substeps=1) as b:
            b.step(300)
            f32.append(b.get_state()[:4])
    assert all(np.array_equal(x, y) for x, y in zip(*f32))


def test_chunked_graphs_match_direct_launches():
    """rod_step(n) on a contact batch replays a graph of 64 one-step launches
    as often as it fits and a graph of the rest (150 = 2 x 64 + 22), bit for
    bit as the same launches made directly, and again on a second call that
    reuses both graphs."""
    import os
    R = _rod()
    inp = _small_pile(seed=99)
    out = []
    for direct in (False, True):
        if direct:
            os.environ["ROD_NO_GRAPH"] = "1"
        try:
            print(f"case: fibre pile 24 rods, 2 x 150 steps, {'direct launches' if direct else 'chunked graphs'}", flush=True)
            with R.RodBatch(inp, precision="f64") as b:
                b.step(150)
                b.step(150)
                out.append(b.get_state()[:4])
        finally:
            if direct:
                del os.environ["ROD_NO_GRAPH"]
    assert all(np.array_equal(x, y) for x, y in zip(*out))
