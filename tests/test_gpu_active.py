"""GPU parity of gravity and the travelling-wave muscle moments (Results,
"Active matter"), alone and together with the magnetic couple, against the
FP64 oracle through the C boundary.  Bars on all five norms as in
test_gpu_step (FP64: 3 x the oracle's one-ulp conditioning; FP32: 4 x its
FP32 mirror's discrepancy), energies (W_ext holding the work of gravity)
included.
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from parity import fp64_bars, oracle_pair, rod_norms
from test_gpu_step import _rod, assert_norms, run_both
from test_gpu_magnetic import _magnetic_edges

pytestmark = pytest.mark.gpu


def _extended_edges(waves, seed=61):
    """The magnetic edge batch (lengths at and around wave and tile edges, both
    clamp types, end forces) with gravity and random muscle waves added."""
    inp = _magnetic_edges(waves, seed)
    rng = np.random.default_rng(seed + 1)
    R = inp.n_rods
    inp.gravity = np.array([0.3, -0.5, -9.81])
    inp.muscle_amp = rng.uniform(-1.0, 1.0, size=inp.n_elements - R) * 1e-4
    inp.muscle_axis = rng.normal(size=(R, 3))
    inp.muscle_freq = rng.uniform(0.0, 30.0, size=R)
    inp.muscle_wavenumber = rng.uniform(-50.0, 50.0, size=R)
    inp.muscle_phase = rng.uniform(0.0, 2 * np.pi, size=R)
    return inp


def test_active_filaments_f64_1000_steps():
    print("case: active filaments 64 rods x 50, gravity + muscle, FP64, 1000 steps", flush=True)
    norms, _ = run_both(W.active_filaments(n_rods=64), 1000)
    assert_norms(norms)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_extended_edges_f64(waves):
    print(f"case: extended edge batch (magnetic + gravity + muscle), tile_waves={waves}, FP64, 300 steps",
          flush=True)
    norms, info = run_both(_extended_edges(waves), 300, tile_waves=waves)
    assert info["tile_waves"] == waves
    assert_norms(norms)


def test_active_f32_parity():
    for name, inp, waves in (("active filaments 64 rods", W.active_filaments(n_rods=64), 0),
                             ("extended edges 8 waves", _extended_edges(8, seed=63), 8)):
        print(f"case: {name}, FP32, 1000 steps", flush=True)
        norms, _ = run_both(inp, 1000, precision="f32", tile_waves=waves)
        assert_norms(norms)


def test_muscle_phase_across_launches():
    """The muscle wave's phase carries over launch and call boundaries (7-step
    launches; 400 + 600 steps) within the FP64 bars of one 1000-step launch."""
    R = _rod()
    inp = W.active_filaments(n_rods=16, period=0.05)
    with R.RodBatch(inp) as b:
        b.step(1000)
        one = b.get_state()
    with R.RodBatch(inp, substeps=7) as b:
        b.step(1000)
        s7 = b.get_state()
    with R.RodBatch(inp) as b:
        b.step(400)
        b.step(600)
        s2 = b.get_state()
    o, pert = oracle_pair(inp, 1000)
    bars, _ = fp64_bars(inp, o, pert, 1000)
    for other in (s7, s2):
        nm = rod_norms(inp, one[:4], other[:4], 1000 * inp.dt)
        bad = {k: (nm[k], bars[k]) for k in nm if not nm[k] <= bars[k]}
        assert not bad, bad


def test_zero_extensions_are_the_plain_step():
    """Zero muscle amplitude, zero magnetization and zero gravity select the
    extended kernel and land on the plain kernel's result bit for bit."""
    R = _rod()
    inp = W.ragged_batch(n_rods=24, n_min=16, n_max=120, seed=49)
    ext = inp.copy()
    ext.muscle_amp = np.zeros(inp.n_elements - inp.n_rods)
    ext.muscle_axis = np.tile([1.0, 0.0, 0.0], (inp.n_rods, 1))
    ext.muscle_freq = np.full(inp.n_rods, 3.0)
    ext.muscle_wavenumber = np.full(inp.n_rods, 10.0)
    ext.muscle_phase = np.zeros(inp.n_rods)
    ext.magnetization = np.zeros((inp.n_elements, 3))
    ext.field = np.full(9, 0.01)
    for prec in ("f64", "f32"):
        with R.RodBatch(inp, precision=prec) as a, R.RodBatch(ext, precision=prec) as b:
            a.step(300)
            b.step(300)
            for x, y in zip(a.get_state()[:4], b.get_state()[:4]):
                assert np.array_equal(x, y)
            assert np.array_equal(a.energy(), b.energy())


def test_active_16384_full_f64_sampled():
    """The benchmark's active batch (16,384 rods x 50, FP64, autotuned), one
    bench step of 1000 steps; 16 seeded rods against the oracle."""
    from test_gpu_fullsize import _full_run
    from parity import energy_norm
    inp = W.active_filaments()
    print("case: active filaments 16,384 rods, f64, 1000 steps, 16-rod oracle sample", flush=True)
    got, e_got, sub, t = _full_run(inp, "f64", 1000, 16, 109)
    o, p = oracle_pair(sub, 1000)
    norms = rod_norms(sub, o.state(), got, 1000 * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_got)
    bars, _ = fp64_bars(sub, o, p, 1000)
    print("norms", {k: f"{v:.2e}" for k, v in norms.items()}, "bars", {k: f"{v:.2e}" for k, v in bars.items()},
          flush=True)
    bad = {k: (norms[k], bars[k]) for k in norms if not norms[k] <= bars[k]}
    assert not bad, bad
