"""Parity at the full workload sizes, in the launch configuration bench.py
times (autotuned tile width and substeps, one rod_step call per bench step):
the GPU advances every rod, the FP64 oracle a seeded sample of them one by one.

Bars on all five norms, as in test_gpu_step: FP64 max(1e-10, 3 x the
oracle's largest one-ulp divergence over three starts); FP32 max(2^-20, 4 x the
discrepancy of the oracle's FP32 mirror over the same steps, 20,000 of them
for the carpets).
"""
import numpy as np
import pytest

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
from parity import check, energy_norm, fp32_bars, fp32_mirror, fp64_bars, oracle_pair, rod_norms
import rodcases as RC
from test_gpu_step import report

pytestmark = pytest.mark.gpu


def _slice_state(inp, state, rods):
    """Rows of the listed rods, in order, from a full-batch state."""
    pos, vel, dr, om = state[:4]
    no, eo, n = inp.node_offset, inp.elem_offset, inp.n_elems
    ni = np.concatenate([np.arange(no[r], no[r] + n[r] + 1) for r in rods])
    ei = np.concatenate([np.arange(eo[r], eo[r] + n[r]) for r in rods])
    return pos[ni], vel[ni], dr[ei], om[ei]


def _full_run(inp, precision, steps, n_sample, seed):
    from paper_2605_13766_amd import rod
    with rod.RodBatch(inp, precision=precision, autotune=True) as b:
        info = b.info()
        b.step(steps)
        state = b.get_state()
        energy = b.energy()
        assert not b.flags().any()
    rods = np.sort(np.random.default_rng(seed).choice(inp.n_rods, size=n_sample, replace=False))
    print(f"tile_waves {info['tile_waves']} substeps {info['substeps']}; sampled rods {rods.tolist()}", flush=True)
    return _slice_state(inp, state, rods), energy[rods], inp.subset(rods), state[4]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_ragged_4096_full_batch_sampled(precision):
    """The benchmark batch (4096 rods, 556,994 elements), one bench step of
    1000 steps; 16 seeded rods against the oracle."""
    inp = W.ragged_batch(n_rods=4096)
    print(f"case: ragged 4096 rods, {precision}, 1000 steps, 16-rod oracle sample", flush=True)
    got, e_got, sub, t = _full_run(inp, precision, 1000, 16, 101)
    assert abs(t - 1000 * inp.dt) < 1e-12
    o, p = oracle_pair(sub, 1000)
    norms = rod_norms(sub, o.state(), got, 1000 * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_got)
    if precision == "f64":
        bars, base = fp64_bars(sub, o, p, 1000)
    else:
        bars, base = fp32_bars(sub, o, fp32_mirror(sub, 1000), 1000)
    report(norms, base, precision)
    bad = check(norms, bars)
    assert not bad, bad


def test_cantilever_full_10000_steps():
    """The single-rod case over its full 10,000 steps (0.1 s): parity with the
    oracle (FP64 bars) and the tip deflection against the Euler-Bernoulli modal
    closed form within 1%."""
    from paper_2605_13766_amd import rod
    inp = W.single_cantilever()
    o, p = oracle_pair(inp, 10000)
    with rod.RodBatch(inp, precision="f64", autotune=True) as b:
        b.step(10000)
        pos, vel, dr, om, t = b.get_state()
        e = b.energy()
    norms = rod_norms(inp, o.state(), (pos, vel, dr, om), t)
    norms["energy"] = energy_norm(o.energy(), e)
    bars, sens = fp64_bars(inp, o, p, 10000)
    report(norms, sens, "f64")
    bad = check(norms, bars)
    assert not bad, bad
    A, I = RC.section(0.01)
    ref = RC.cantilever_modal_tip(t, 1e-3, 1e6, I, 1000.0, A, 1.0)
    tip = -pos[-1, 2]
    print("tip deflection", tip, "modal closed form", ref, "total energy", e.sum())
    assert abs(tip / ref - 1) < 0.01


def full_f32_against_mirror(inp, steps, n_sample, seed):
    """Full-size FP32 run; a seeded sample of rods against the FP64 oracle,
    all five norms within the FP32 bars of the mirror's own discrepancy."""
    got, e_got, sub, t = _full_run(inp, "f32", steps, n_sample, seed)
    o = ro.Oracle(sub)
    o.step(steps)
    norms = rod_norms(sub, o.state(), got, steps * inp.dt)
    norms["energy"] = energy_norm(o.energy(), e_got)
    bars, base = fp32_bars(sub, o, fp32_mirror(sub, steps), steps)
    report(norms, base, "f32")
    bad = check(norms, bars)
    assert not bad, bad


def test_carpet_65536_full_f32_20000_steps():
    """The cilia carpet (65,536 rods x 50, FP32, autotuned) over its full
    20,000 steps; 64 seeded rods against the FP64 oracle.  The FP32 mirror
    itself departs from the FP64 oracle by about 3e-2 in omega and 1e-3 in
    velocity over these steps (the stiff shear modes carry FP32 round-off):
    that is the scale the bar follows."""
    inp = W.cilia_carpet()
    print("case: carpet 65,536 rods, f32, 20,000 steps, 64-rod oracle sample", flush=True)
    full_f32_against_mirror(inp, 20000, 64, 103)
