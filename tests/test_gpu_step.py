"""GPU parity of the rod step (through the C boundary) against the FP64 oracle.

Bars per norm (tests/parity.py), on all five norms in both precisions:
FP64 max(1e-10, 3 x the oracle's own largest divergence over three starts
whose positions move by one ulp); positions, velocities and directors sit
orders below 1e-10, while the angular velocity of these stiff rods is
conditioned at a few 1e-10 after 1000 steps, which is where the GPU lands as
well.  FP32 max(2^-20, 4 x the discrepancy of the oracle's FP32 mirror).
"""
import numpy as np
import pytest

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
from parity import bars_for, check, energy_norm, fp64_bars, oracle_pair, rod_norms
import rodcases as RC

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _rod():
    from paper_2605_13766_amd import rod
    return rod


def report(norms, base, precision):
    """Print the norms, what the bars derive from, and each norm's ratio to it."""
    what = "1-ulp conditioning" if precision == "f64" else "FP32 mirror discrepancy"
    print("norms", {k: f"{v:.2e}" for k, v in norms.items() if k in base}, flush=True)
    print(what, {k: f"{v:.2e}" for k, v in base.items()}, flush=True)
    print("ratio", {k: f"{norms[k] / v:.2f}" if v > 0 else "-" for k, v in base.items()}, flush=True)


def run_both(inp, steps, precision="f64", **kw):
    R = _rod()
    o, bars, base = bars_for(inp, precision, steps)
    with R.RodBatch(inp, precision=precision, **kw) as b:
        b.step(steps)
        pos, vel, dr, om, t = b.get_state()
        e_gpu = b.energy()
        info = b.info()
    assert abs(t - steps * inp.dt) < 1e-12 * max(1.0, steps * inp.dt)
    norms = rod_norms(inp, o.state(), (pos, vel, dr, om), steps * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_gpu)
    report(norms, base, precision)
    norms["bars"] = bars
    return norms, info


def assert_norms(norms, keys=("pos", "vel", "dir", "omega", "energy")):
    bad = check(norms, norms["bars"], keys)
    assert not bad, f"norms above their bars: {bad}"


def test_cantilever_f64_1000_steps():
    print("case: cantilever 100 elements, FP64, 1000 steps", flush=True)
    norms, _ = run_both(W.single_cantilever(), 1000)
    assert_norms(norms)


def test_ragged_sample_f64_1000_steps():
    print("case: ragged batch 64 rods (16..256 elements), FP64, 1000 steps", flush=True)
    inp = W.ragged_batch(n_rods=64)
    norms, info = run_both(inp, 1000)
    assert info["tile_waves"] == 4
    assert_norms(norms)


def test_carpet_sample_f64_couple():
    print("case: carpet 64 rods x 50, driven couple, FP64, 1000 steps", flush=True)
    inp = W.cilia_carpet(grid=8, dt=1e-6)
    norms, _ = run_both(inp, 1000)
    assert_norms(norms)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_edge_lengths_and_boundaries(waves):
    """Rod lengths at and around tile and wave edges, both clamp types, end
    forces and couples, in one ragged batch."""
    print(f"case: edge batch, tile_waves={waves}", flush=True)
    rng = np.random.default_rng(21)
    cap = 64 * waves
    lengths = [1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 511, 512]
    lengths = [n for n in lengths if n <= cap]
    nodes_list, Q_list, vel_list, om_list = [], [], [], []
    for n in lengths:
        nodes = W._fourier_curve(rng, 0.01 * n, n, 3.0) if n >= 2 else np.array([[0, 0, 0], [0.01, 0, 0.0]])
        nodes_list.append(nodes)
        Q_list.append(W.frames_parallel_transport(nodes))
        vel_list.append(rng.normal(0, 1e-3, size=(n + 1, 3)))
        om_list.append(rng.normal(0, 0.1, size=(n, 3)))
    R = len(lengths)
    inp = W._assemble("edges", nodes_list, Q_list, 1e-5, density=1000.0,
                      youngs=10 ** rng.uniform(5, 7, R), radius=rng.uniform(0.005, 0.02, R),
                      damping=rng.uniform(0, 0.5, R), bc_start=rng.integers(0, 2, R),
                      bc_end=rng.integers(0, 2, R), velocity_list=vel_list, omega_list=om_list,
                      end_force=rng.normal(0, 1e-3, (R, 3)), couple_amp=rng.normal(0, 1e-4, (R, 3)),
                      couple_freq=rng.uniform(0, 20, R), couple_phase=rng.uniform(0, 6.28, R))
    norms, info = run_both(inp, 300, tile_waves=waves)
    assert info["tile_waves"] == waves
    assert_norms(norms)


def test_tile_layout_bitwise_invariant():
    """The packed layout does not change any result bit: same batch, four tile widths."""
    R = _rod()
    inp = W.ragged_batch(n_rods=24, n_min=16, n_max=60, seed=31)
    outs = []
    for waves in (1, 2, 4, 8):
        with R.RodBatch(inp, tile_waves=waves) as b:
            b.step(200)
            outs.append(b.get_state()[:4])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_autotuner_keeps_the_fastest_and_the_results():
    """autotune: every fitting tile width (rods of up to 100 elements: 2, 4
    and 8 waves) times substeps 50 / 200 / 1000 is timed; the batch uses the
    fastest; its results equal those of a batch created with that choice by
    hand, bit for bit, and of the same substeps at another tile width."""
    R = _rod()
    inp = W.ragged_batch(n_rods=512, n_min=16, n_max=100, seed=37)
    with R.RodBatch(inp, autotune=True) as b:
        trials = b.tuning()
        info = b.info()
        print(trials, info)
        assert sorted((t["tile_waves"], t["substeps"]) for t in trials) == \
            [(w, s) for w in (2, 4, 8) for s in (50, 200, 1000)]
        assert all(t["ns_per_element_step"] > 0 for t in trials)
        best = min(trials, key=lambda t: t["ns_per_element_step"])
        assert (info["tile_waves"], info["substeps"]) == (best["tile_waves"], best["substeps"])
        b.step(600)
        got = b.get_state()
    other = 2 if info["tile_waves"] != 2 else 4
    for w in (info["tile_waves"], other):
        with R.RodBatch(inp, tile_waves=w, substeps=info["substeps"]) as c:
            assert c.tuning() == []
            c.step(600)
            ref = c.get_state()
        for a, r in zip(got[:4], ref[:4]):
            assert np.array_equal(a, r)


def test_resume_bitwise_and_launch_split_roundoff():
    """Checkpoint/resume at a launch boundary is bitwise: 500 steps, get_state,
    a fresh batch set_state, 500 steps == 500 + 500 steps in one batch.  A
    different launch partition (400 + 600 steps, or 7-step launches) fuses
    different half drifts, so it agrees with one 1000-step launch to round-off:
    within the FP64 parity bars."""
    R = _rod()
    inp = W.ragged_batch(n_rods=16, n_min=16, n_max=100, seed=33)
    with R.RodBatch(inp) as b:
        b.step(500)
        p, v, d, w, t = b.get_state()
        b.step(500)
        ref_split = b.get_state()
    with R.RodBatch(inp) as b:
        b.set_state(p, v, d, w, t)
        b.step(500)
        resumed = b.get_state()
    for a, c in zip(ref_split[:4], resumed[:4]):
        assert np.array_equal(a, c)
    assert abs(resumed[4] - ref_split[4]) < 1e-15
    with R.RodBatch(inp) as b:
        b.step(1000)
        one = b.get_state()
    with R.RodBatch(inp) as b:
        b.step(400)
        b.step(600)
        s2 = b.get_state()
    with R.RodBatch(inp, substeps=7) as b:
        b.step(1000)
        s3 = b.get_state()
    o, pert = oracle_pair(inp, 1000)
    bars, _ = fp64_bars(inp, o, pert, 1000)
    for other in (s2, s3, ref_split):
        nm = rod_norms(inp, one[:4], other[:4], 1000 * inp.dt)
        bad = {k: (nm[k], bars[k]) for k in nm if not nm[k] <= bars[k]}
        assert not bad, bad


def test_graph_replay_repeatable():
    """Replaying the captured graph advances exactly like direct launches."""
    R = _rod()
    inp = W.ragged_batch(n_rods=8, n_min=16, n_max=80, seed=35)
    with R.RodBatch(inp) as b:
        for _ in range(5):
            b.step(100)          # same n_steps: one capture, four replays
        a = b.get_state()
    import os
    os.environ["ROD_NO_GRAPH"] = "1"
    try:
        with R.RodBatch(inp) as b:
            for _ in range(5):
                b.step(100)
            c = b.get_state()
    finally:
        del os.environ["ROD_NO_GRAPH"]
    for x, y in zip(a[:4], c[:4]):
        assert np.array_equal(x, y)


def test_energy_matches_oracle_at_start():
    R = _rod()
    inp = W.ragged_batch(n_rods=32, seed=37)
    o = ro.Oracle(inp)
    with R.RodBatch(inp) as b:
        e = b.energy()
    ref = o.energy()
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.all(np.abs(e - ref) <= 1e-12 * scale + 1e-300)


def test_nonfinite_flag_raised():
    """A time step far above the stability limit drives the state to NaN/Inf:
    the kernel flags the rod and the synchronising calls report it."""
    R = _rod()
    inp = W.ragged_batch(n_rods=4, n_min=16, n_max=32, seed=39)
    inp.dt = 1e-2
    with R.RodBatch(inp) as b:
        assert "stability" in b.warning
        b.step(2000)
        f = b.flags()
        assert f.sum() >= 1
        with pytest.raises(R.RodError) as ei:
            b.energy()
        assert ei.value.code == R.ROD_ENONFINITE


def test_f32_parity():
    """FP32 state (edge-vector form) against the FP64 oracle, 1000 steps, all
    five norms within 4 x the FP32 mirror's discrepancy."""
    for name, inp in (("ragged 64 rods", W.ragged_batch(n_rods=64)),
                      ("carpet 64 rods", W.cilia_carpet(grid=8, dt=1e-6))):
        print(f"case: {name}, FP32, 1000 steps", flush=True)
        norms, _ = run_both(inp, 1000, precision="f32")
        assert_norms(norms)


def test_device_inputs_give_the_same_batch():
    """inputs_on_device = 1 (every input a device array) builds the same batch
    as host inputs: identical state after creation and after 100 steps."""
    R = _rod()
    inp = W.ragged_batch(n_rods=24, n_min=16, n_max=120, seed=43)
    for prec in ("f64", "f32"):
        with R.RodBatch(inp, precision=prec) as a, R.RodBatch(inp, precision=prec, device_inputs=True) as b:
            for x, y in zip(a.get_state()[:4], b.get_state()[:4]):
                assert np.array_equal(x, y)
            a.step(100)
            b.step(100)
            for x, y in zip(a.get_state()[:4], b.get_state()[:4]):
                assert np.array_equal(x, y)


def test_zero_and_negative_steps():
    """rod_step(0) is a no-op (state and time bit for bit), a negative count is
    ROD_EINVAL, and a contact batch behaves the same."""
    print("case: zero and negative step counts, plain and contact batches", flush=True)
    R = _rod()
    for inp in (W.ragged_batch(n_rods=8, n_min=16, n_max=40, seed=3),
                W.fibre_pile(n_rods=8, n=10, L=0.1, per_row=2, rows=2)):
        with R.RodBatch(inp, precision="f64") as b:
            b.step(3)
            before = b.get_state()
            b.step(0)
            after = b.get_state()
            for x, y in zip(before[:4], after[:4]):
                assert np.array_equal(x, y)
            assert before[4] == after[4]
            with pytest.raises(R.RodError) as ei:
                b.step(-1)
            assert ei.value.code == R.ROD_EINVAL
