"""Pins of the oracle's FP32 mirror (CPU): it computes in single precision
(its state is FP32 and departs from the FP64 oracle by FP32-sized amounts that
shrink when FP64 is used), it holds what FP32 can hold of the exact
equilibria, and its edge form keeps a rest rod at rest far from the origin,
where absolute FP32 positions could not."""
import numpy as np

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
from parity import energy_norm, rod_norms
import rodcases as RC


def test_mirror_is_single_precision_and_close_to_fp64():
    inp = W.ragged_batch(n_rods=6, n_min=16, n_max=60, seed=11)
    o, m = ro.Oracle(inp), ro.Oracle32(inp)
    for a in (m.x, m.vel, m.dir, m.omega):
        assert a.dtype == np.float32
    o.step(500)
    m.step(500)
    nm = rod_norms(inp, o.state(), m.state(), 500 * inp.dt)
    nm["energy"] = energy_norm(o.energy(), m.energy())
    # FP32-sized, not FP64-sized and not broken: 2^-24 = 6e-8 per operation,
    # accumulated over 500 steps of stiff rods
    assert 1e-9 < nm["pos"] < 1e-5 and 1e-8 < nm["dir"] < 1e-4, nm
    assert nm["vel"] < 1e-4 and nm["omega"] < 1e-2 and nm["energy"] < 1e-3, nm


def test_mirror_step_matches_oracle_at_start():
    """One step from the same start: the mirror's result is the oracle's
    rounded to FP32 up to a few FP32 rounding units of each field's scale."""
    inp = W.cilia_carpet(grid=2, dt=1e-6)
    o, m = ro.Oracle(inp), ro.Oracle32(inp)
    o.step(1)
    m.step(1)
    for a, b in zip(o.state(), m.state()):
        scale = max(np.abs(a).max(), 1e-30)
        assert np.abs(a - b).max() <= 64 * 2.0 ** -24 * scale


def test_mirror_rest_rod_far_from_origin_stays_at_rest():
    """A straight unstretched rod at rest 100 m from the origin, no loads: in
    FP32 absolute coordinates its 1 cm elements would be resolved only to
    7.6e-6 m; the mirror's edge form keeps every node within 1e-9 m of where
    it started after 1000 steps (the rounded rest lengths and edges leave
    strains of order 1e-7, which barely move it)."""
    n, L = 50, 0.5
    nodes, Q = RC.twisted_rod(n, L, 0.0)
    nodes = nodes + np.array([100.0, -100.0, 100.0])
    inp = RC.single(nodes, Q, E=1e6, radius=0.01)
    m = ro.Oracle32(inp)
    start = m.state()[0]      # the edges rounded once to FP32
    assert np.abs(start - nodes).max() < n * 2.0 ** -24 * (L / n)
    m.step(1000)
    pos = m.state()[0]
    assert np.abs(pos - start).max() < 1e-9


def test_mirror_clamped_ends_hold():
    """Both clamps of the mirror: node 0 stays exactly at its initial
    position (its anchor is 0), node n within the FP32 rounding of the last
    edge (which is set so that node n sits there), and their elements keep
    their frames."""
    inp = W.ragged_batch(n_rods=3, n_min=20, n_max=30, seed=13)
    inp.bc_start[:] = 1
    inp.bc_end[:] = 1
    m = ro.Oracle32(inp)
    m.step(300)
    pos, _, dr, _ = m.state()
    no, eo, ne = inp.node_offset, inp.elem_offset, inp.n_elems
    for r in range(inp.n_rods):
        j0, jn = no[r], no[r] + ne[r]
        assert np.array_equal(pos[j0], inp.position[j0])
        last = np.linalg.norm(inp.position[jn] - inp.position[jn - 1])
        assert np.abs(pos[jn] - inp.position[jn]).max() <= 2.0 ** -24 * last + 1e-15 * np.abs(pos[jn]).max()
        for i in (eo[r], eo[r] + ne[r] - 1):
            assert np.array_equal(dr[i], inp.director[i].astype(np.float32).astype(np.float64))
