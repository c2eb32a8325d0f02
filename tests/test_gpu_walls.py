"""GPU parity of planar walls (penalty contact per node, damping proportional
to the penetration, regularised Coulomb friction) against the FP64 oracle through the C boundary,
alone and with connections.  Bars on all five norms as in test_gpu_step (FP64:
3 x the oracle's one-ulp conditioning; FP32: 4 x its FP32 mirror's
discrepancy), energies (W_ext holding the penalty potential) included.
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from parity import energy_norm, fp64_bars, oracle_pair, rod_norms
from test_gpu_step import _rod, assert_norms, run_both

pytestmark = pytest.mark.gpu


def _boxed(waves, seed=81):
    """Curved rods of lengths up to a tile of `waves` waves in a 0.6 m box,
    every third starting pressed into the floor by half its radius, the
    others moving toward the walls, under gravity with friction; both clamp
    types.  Parameters keep the explicit step stable: contact frequency
    sqrt(k/m) h and friction rate mu f_n h / (m v_slip) well below 2."""
    rng = np.random.default_rng(seed)
    cap = 64 * waves
    lengths = [n for n in (1, 2, 3, 31, 63, 64, 65, 127, 128, 129, 200, 255, 256, 400, 511, 512) if n <= cap]
    nodes_list, Q_list, vel_list = [], [], []
    box, rad = 0.6, 0.003
    for k, n in enumerate(lengths):
        ds = min(0.01, 0.5 / max(n, 1))
        nodes = W._fourier_curve(rng, ds * max(n, 2), max(n, 2), 3.0)[: n + 1] if n >= 2 else \
            np.array([[0, 0, 0], [ds, 0, 0.0]])
        nodes = nodes - nodes.min(axis=0)
        span = nodes.max(axis=0)
        if k % 3 == 0:
            nodes = nodes + np.array([0.01, 0.01, 0.5 * rad])
        else:
            nodes = nodes + 0.01 + rng.uniform(0, 1, 3) * np.maximum(box - 0.02 - span, 0.0)
        nodes_list.append(nodes)
        Q_list.append(W.frames_parallel_transport(nodes))
        vel_list.append(np.tile(rng.normal(0, 0.2, 3), (n + 1, 1)) + rng.normal(0, 1e-3, (n + 1, 3)))
    R = len(lengths)
    inp = W._assemble("boxed", nodes_list, Q_list, 2e-6, density=1000.0, youngs=10 ** rng.uniform(5, 6.5, R),
                      radius=np.full(R, rad), damping=rng.uniform(0, 0.5, R), bc_start=rng.integers(0, 2, R),
                      bc_end=np.zeros(R, np.int32), velocity_list=vel_list)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.walls = np.array([[0, 0, 1, 0], [1, 0, 0, 0], [-1, 0, 0, -box], [0, 1, 0, 0], [0, -1, 0, -box],
                          [0, 0, -1, -box]], float)
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 200.0, 200.0, 0.4, 0.05
    return inp


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_boxed_rods_f64(waves):
    print(f"case: rods in a walled box, tile_waves={waves}, FP64, 1000 steps", flush=True)
    norms, info = run_both(_boxed(waves), 1000, tile_waves=waves)
    assert info["tile_waves"] == waves
    assert_norms(norms)


def test_walls_with_connections_f64():
    print("case: 4 millipede bots on a floor, FP64, 1000 steps", flush=True)
    inp = W.millipede_swarm(n_bots=4)
    inp.position[:, 2] += 0.0045 - inp.position[:, 2].min()   # lowest leg tip just above the floor
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.walls = np.array([[0.0, 0.0, 1.0, 0.0]])
    inp.wall_k, inp.wall_c, inp.wall_mu, inp.wall_vslip = 5.0, 50.0, 0.5, 1e-4
    norms, _ = run_both(inp, 1000)
    assert_norms(norms)


def test_walls_f32_parity():
    for name, inp, waves in (("boxed rods 4 waves", _boxed(4, seed=83), 4),
                             ("active box 64 rods", W.active_filaments(n_rods=64, box=True), 0)):
        print(f"case: {name}, FP32, 1000 steps", flush=True)
        norms, _ = run_both(inp, 1000, precision="f32", tile_waves=waves)
        assert_norms(norms)


def test_active_box_full_f64_sampled():
    """The active filaments in the 2L box (16,384 rods, FP64, autotuned) over
    4000 steps (0.2 s, the rods reach the floor); 16 seeded rods against the oracle."""
    from test_gpu_fullsize import _full_run
    inp = W.active_filaments(box=True)
    print("case: active box 16,384 rods, f64, 4000 steps, 16-rod oracle sample", flush=True)
    got, e_got, sub, t = _full_run(inp, "f64", 4000, 16, 113)
    o, p = oracle_pair(sub, 4000)
    norms = rod_norms(sub, o.state(), got, 4000 * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_got)
    bars, _ = fp64_bars(sub, o, p, 4000)
    print("norms", {k: f"{v:.2e}" for k, v in norms.items()}, "bars", {k: f"{v:.2e}" for k, v in bars.items()},
          flush=True)
    bad = {k: (norms[k], bars[k]) for k in norms if not norms[k] <= bars[k]}
    assert not bad, bad


def test_eight_walls_f64():
    """The largest wall count (ROD_MAX_WALLS = 8): the box's six walls and two
    slanted ones cutting its lower corners, so that every slot of the kernel's
    wall table is in use and some rods touch a slanted wall."""
    print("case: rods in a box with 8 walls (2 slanted), tile_waves=4, FP64, 1000 steps", flush=True)
    inp = _boxed(4, seed=85)
    s2 = np.sqrt(0.5)
    rad = np.repeat(inp.radius, inp.n_elems + 1)
    slanted = []
    for n in ([s2, s2, 0.0], [-s2, s2, 0.0]):
        # placed so that the nearest node starts 0.5 mm into it
        gap = inp.position @ np.array(n) - rad
        slanted.append(n + [gap.min() + 5e-4])
    inp.walls = np.concatenate([inp.walls, np.array(slanted)])
    assert len(inp.walls) == 8
    norms, _ = run_both(inp, 1000, tile_waves=4)
    assert_norms(norms)
