"""GPU parity of rod-rod connections (Results, "Magnetized filament
assemblies"; central spring-dashpots between node pairs, rods joined by them
packed into one tile) against the FP64 oracle through the C boundary.  Bars on
all five norms as in test_gpu_step (FP64: 3 x the oracle's one-ulp
conditioning; FP32: 4 x its FP32 mirror's discrepancy), energies (W_ext
holding half of each spring's potential) included.
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from parity import energy_norm, fp64_bars, oracle_pair, rod_norms
from test_gpu_step import _rod, assert_norms, run_both

pytestmark = pytest.mark.gpu


def _linked(waves, seed=71):
    """Groups of two or three curved rods that fit a tile of `waves` waves,
    joined at interior nodes, at node 0 and at node n, with a connection between
    two nodes of the same rod and one between initially coincident nodes;
    random velocities, both clamp types, gravity."""
    rng = np.random.default_rng(seed)
    cap = 64 * waves
    nodes_list, Q_list, vel_list, om_list = [], [], [], []
    conn_rod, conn_node, rest = [], [], []
    groups = 0
    while groups < 4:
        sizes = rng.integers(1, max(2, cap // 3), size=int(rng.integers(2, 4)))
        if sizes.sum() > cap:
            continue
        first = len(nodes_list)
        for k, n in enumerate(sizes):
            n = int(n)
            nodes = W._fourier_curve(rng, 0.01 * max(n, 2), max(n, 2), 3.0)[: n + 1] if n >= 2 else \
                np.array([[0, 0, 0], [0.01, 0, 0.0]])
            if k == 0:
                nodes = nodes + np.array([0.05 * groups, 0.0, 0.0])
            else:   # chained: node 0 on the previous rod's node n (exactly, for the first link)
                prev = nodes_list[-1][-1]
                nodes = nodes - nodes[0] + prev + (0.0 if k == 1 else np.array([0.0, 0.003, 0.0]))
            nodes_list.append(nodes)
            Q_list.append(W.frames_parallel_transport(nodes))
            vel_list.append(rng.normal(0, 1e-3, size=(n + 1, 3)))
            om_list.append(rng.normal(0, 0.1, size=(n, 3)))
        ids = list(range(first, len(nodes_list)))
        for a, b in zip(ids[:-1], ids[1:]):
            na, nb = int(sizes[a - first]), int(sizes[b - first])
            for (ia, ib) in ((na, 0), (int(rng.integers(0, na + 1)), int(rng.integers(0, nb + 1)))):
                conn_rod.append([a, b]); conn_node.append([ia, ib])
                rest.append(np.linalg.norm(nodes_list[b][ib] - nodes_list[a][ia]) * rng.uniform(0.8, 1.2))
            rest[-2] = 0.0 if b == first + 1 else rest[-2]   # the exact end-to-end link: rest 0
        if sizes[0] >= 3:   # two nodes of one rod, and a coincident pair (rest 0, zero length at start)
            conn_rod.append([first, first]); conn_node.append([0, int(sizes[0])]); rest.append(0.005)
        groups += 1
    R = len(nodes_list)
    inp = W._assemble("linked", nodes_list, Q_list, 1e-5, density=1000.0,
                      youngs=10 ** rng.uniform(5, 6.5, R), radius=rng.uniform(0.005, 0.01, R),
                      damping=rng.uniform(0, 0.5, R), bc_start=rng.integers(0, 2, R),
                      bc_end=rng.integers(0, 2, R), velocity_list=vel_list, omega_list=om_list)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    inp.conn_rod = np.array(conn_rod, np.int32)
    inp.conn_node = np.array(conn_node, np.int32)
    C = len(conn_rod)
    inp.conn_k = rng.uniform(0.5, 5.0, C)
    inp.conn_c = rng.uniform(0.0, 1e-3, C)
    inp.conn_rest = np.array(rest)
    return inp


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_linked_groups_f64(waves):
    print(f"case: linked rod groups, tile_waves={waves}, FP64, 300 steps", flush=True)
    norms, info = run_both(_linked(waves), 300, tile_waves=waves)
    assert info["tile_waves"] == waves
    assert_norms(norms)


def test_millipede_bots_f64_1000_steps():
    print("case: 4 millipede bots (26 rods, 232 elements, 45 connections each), FP64, 1000 steps", flush=True)
    norms, info = run_both(W.millipede_swarm(n_bots=4), 1000)
    assert info["tile_waves"] == 4
    assert_norms(norms)


def test_connections_f32_parity():
    for name, inp, waves in (("millipede 4 bots", W.millipede_swarm(n_bots=4), 0),
                             ("linked groups 2 waves", _linked(2, seed=73), 2)):
        print(f"case: {name}, FP32, 1000 steps", flush=True)
        norms, _ = run_both(inp, 1000, precision="f32", tile_waves=waves)
        assert_norms(norms)


def test_connected_group_kept_in_one_tile_and_too_big_rejected():
    R = _rod()
    inp = W.millipede_swarm(n_bots=1)
    with pytest.raises(R.RodError) as ei:
        R.RodBatch(inp, tile_waves=2)
    assert ei.value.code == R.ROD_EUNSUPPORTED
    big = W.millipede_swarm(n_bots=1, n_back=100, legs_per_side=20)
    with pytest.raises(R.RodError) as ei:
        R.RodBatch(big)
    assert ei.value.code == R.ROD_EUNSUPPORTED


def test_millipede_swarm_full_sampled():
    """224 bots (5,824 rods, 10,080 connections) as bench.py times them: FP64,
    autotuned, one bench step of 1000 steps; 4 seeded bots against the oracle."""
    R = _rod()
    inp = W.millipede_swarm()
    per_bot = inp.n_rods // 224
    with R.RodBatch(inp, precision="f64", autotune=True) as b:
        info = b.info()
        b.step(1000)
        pos, vel, dr, om, t = b.get_state()
        e_gpu = b.energy()
        assert not b.flags().any()
    bots = np.sort(np.random.default_rng(111).choice(224, size=4, replace=False))
    rods = np.concatenate([np.arange(k * per_bot, (k + 1) * per_bot) for k in bots])
    print(f"tile_waves {info['tile_waves']} substeps {info['substeps']}; bots {bots.tolist()}", flush=True)
    sub = inp.subset(rods)
    no, eo, n = inp.node_offset, inp.elem_offset, inp.n_elems
    ni = np.concatenate([np.arange(no[r], no[r] + n[r] + 1) for r in rods])
    ei = np.concatenate([np.arange(eo[r], eo[r] + n[r]) for r in rods])
    o, p = oracle_pair(sub, 1000)
    norms = rod_norms(sub, o.state(), (pos[ni], vel[ni], dr[ei], om[ei]), 1000 * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_gpu[rods])
    bars, _ = fp64_bars(sub, o, p, 1000)
    print("norms", {k: f"{v:.2e}" for k, v in norms.items()}, "bars", {k: f"{v:.2e}" for k, v in bars.items()},
          flush=True)
    bad = {k: (norms[k], bars[k]) for k in norms if not norms[k] <= bars[k]}
    assert not bad, bad
