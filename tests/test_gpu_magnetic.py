"""GPU parity of the magnetic couple (Methods, "Magnetized filaments", Eq. 2:
c_mag = m x (Q b(t)) joins the couple of Eq. 1b) against the FP64 oracle,
through the C boundary.  Bars on all five norms as in test_gpu_step (FP64: 3 x the
oracle's one-ulp conditioning; FP32: 4 x its FP32 mirror's discrepancy).
"""
import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W
from parity import fp64_bars, oracle_pair, rod_norms
from test_gpu_step import _rod, assert_norms, run_both

pytestmark = pytest.mark.gpu


def _magnetic_edges(waves, seed=51):
    """Rods at and around wave and tile edges, both clamp types, random
    per-element magnetization, a static plus rotating field and an end force."""
    rng = np.random.default_rng(seed)
    cap = 64 * waves
    lengths = [n for n in (1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 511, 512) if n <= cap]
    nodes_list, Q_list, vel_list, om_list = [], [], [], []
    for n in lengths:
        nodes = W._fourier_curve(rng, 0.01 * n, n, 3.0) if n >= 2 else np.array([[0, 0, 0], [0.01, 0, 0.0]])
        nodes_list.append(nodes)
        Q_list.append(W.frames_parallel_transport(nodes))
        vel_list.append(rng.normal(0, 1e-3, size=(n + 1, 3)))
        om_list.append(rng.normal(0, 0.1, size=(n, 3)))
    R = len(lengths)
    inp = W._assemble("magnetic_edges", nodes_list, Q_list, 1e-5, density=1000.0,
                      youngs=10 ** rng.uniform(5, 7, R), radius=rng.uniform(0.005, 0.02, R),
                      damping=rng.uniform(0, 0.5, R), bc_start=rng.integers(0, 2, R),
                      bc_end=rng.integers(0, 2, R), velocity_list=vel_list, omega_list=om_list,
                      end_force=rng.normal(0, 1e-3, (R, 3)))
    inp.magnetization = rng.normal(0, 0.5, size=(inp.n_elements, 3))
    inp.field = rng.normal(0, 0.02, size=9)
    inp.field_freq = 37.0
    return inp


def test_magnetic_carpet_f64_1000_steps():
    print("case: magnetic carpet 64 rods x 50, FP64, 1000 steps", flush=True)
    norms, _ = run_both(W.magnetic_carpet(grid=8), 1000)
    assert_norms(norms)


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_magnetic_edges_f64(waves):
    print(f"case: magnetic edge batch, tile_waves={waves}, FP64, 300 steps", flush=True)
    norms, info = run_both(_magnetic_edges(waves), 300, tile_waves=waves)
    assert info["tile_waves"] == waves
    assert_norms(norms)


def test_magnetic_f32_parity():
    for name, inp, waves in (("magnetic carpet 64 rods", W.magnetic_carpet(grid=8), 0),
                             ("magnetic edges 8 waves", _magnetic_edges(8, seed=53), 8)):
        print(f"case: {name}, FP32, 1000 steps", flush=True)
        norms, _ = run_both(inp, 1000, precision="f32", tile_waves=waves)
        assert_norms(norms)


def test_field_phase_across_launches():
    """The field's phase carries over launch and call boundaries: 7-step
    launches, and 400 + 600 steps in two calls, agree with one 1000-step
    launch within the FP64 bars (they differ only in the fused half drifts)."""
    R = _rod()
    inp = W.magnetic_carpet(grid=4, freq=50.0)
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


def test_zero_magnetization_is_the_plain_step():
    """A batch with zero magnetization runs the magnetic kernel and lands on
    the plain kernel's result bit for bit, in both precisions."""
    R = _rod()
    inp = W.ragged_batch(n_rods=24, n_min=16, n_max=120, seed=47)
    mag = inp.copy()
    mag.magnetization = np.zeros((inp.n_elements, 3))
    mag.field = np.full(9, 0.01)
    mag.field_freq = 5.0
    for prec in ("f64", "f32"):
        with R.RodBatch(inp, precision=prec) as a, R.RodBatch(mag, precision=prec) as b:
            a.step(300)
            b.step(300)
            for x, y in zip(a.get_state()[:4], b.get_state()[:4]):
                assert np.array_equal(x, y)


def test_surrogate_rejects_magnetic_batches():
    R = _rod()
    inp = W.magnetic_carpet(grid=2, n=64)
    import torch
    with R.RodBatch(inp, precision="f32") as b, R.Surrogate(k_substeps=32) as s:
        out = torch.zeros((s.n_windows(b), 96), dtype=torch.float32, device="cuda")
        with pytest.raises(R.RodError) as ei:
            s.features(b, out)
        assert ei.value.code == R.ROD_EUNSUPPORTED and "magnetic" in str(ei.value)


def test_magnetic_carpet_65536_full_f32_20000_steps():
    """The magnetic carpet at full size (65,536 rods x 50, FP32, autotuned, as
    bench.py times it) over 20,000 steps (a fifth of a field period); 64 seeded rods
    against the FP64 oracle, FP32 bars from the mirror over the same steps."""
    from test_gpu_fullsize import full_f32_against_mirror
    inp = W.magnetic_carpet()
    print("case: magnetic carpet 65,536 rods, f32, 20,000 steps, 64-rod oracle sample", flush=True)
    full_f32_against_mirror(inp, 20000, 64, 107)
