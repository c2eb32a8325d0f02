"""rod_energy_noalloc (energies staged in the library's static device buffer)
against rod_energy (staged in memory allocated with the batch): the same
kernels on the same state, so the results must agree bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2605_13766_amd import workloads as W

pytestmark = pytest.mark.gpu


def _vertical_rods(R, n=2, L=0.01):
    """R free straight rods of n elements along +z on a square grid, node
    velocities N(0, 1e-3^2) m/s (vectorised)."""
    side = int(np.ceil(np.sqrt(R)))
    k = np.arange(R)
    base = np.stack([(k % side) * 2.5e-3, (k // side) * 2.5e-3, np.zeros(R)], axis=1)
    z = np.linspace(0.0, L, n + 1)
    pos = (base[:, None, :] + z[None, :, None] * np.array([0.0, 0.0, 1.0])).reshape(-1, 3)
    vel = np.random.default_rng(R).normal(0.0, 1e-3, size=pos.shape)
    Q = np.broadcast_to(np.eye(3), (R * n, 3, 3)).copy()
    one = np.ones(R)
    return W.RodInputs(
        n_elems=np.full(R, n, np.int32), position=pos, velocity=vel, director=Q,
        omega=np.zeros((R * n, 3)), density=1000.0 * one, youngs=1e6 * one, shear_modulus=1e6 / 1.5 * one,
        radius=2e-4 * one, shear_coeff=4.0 / 3.0 * one, damping=0.0 * one,
        bc_start=np.zeros(R, np.int32), bc_end=np.zeros(R, np.int32), dt=1e-6, name="vertical rods")


def _both(b):
    a = b.energy()
    c = b.energy_noalloc()
    print(f"{b.n_rods} rods: max |E| {np.abs(a).max():.3e}, equal {np.array_equal(a, c)}", flush=True)
    return a, c


def test_noalloc_energy_matches_rod_energy_on_two_calls_the_second_smaller():
    from paper_2605_13766_amd import rod
    print("case: ragged 256 rods FP64 (200 steps), then ragged 8 rods FP32 (100 steps)", flush=True)
    big = rod.RodBatch(W.ragged_batch(n_rods=256, n_min=16, n_max=200, seed=W.SEED_BASE + 41), precision="f64")
    big.step(200)
    a, c = _both(big)
    assert np.array_equal(a, c)
    small = rod.RodBatch(W.ragged_batch(n_rods=8, n_min=16, n_max=60, seed=W.SEED_BASE + 42), precision="f32")
    small.step(100)
    a2, c2 = _both(small)
    assert c2.shape == (8, 5) and np.array_equal(a2, c2)
    # the larger batch again after the smaller one overwrote the front of the buffer
    a3, c3 = _both(big)
    assert np.array_equal(a3, c3) and np.array_equal(a3, a)
    big.close()
    small.close()


def test_noalloc_energy_with_rod_contact_and_walls():
    from paper_2605_13766_amd import rod
    print("case: fibre pile 24 rods x 20 with contact and a floor, FP64, 300 steps", flush=True)
    inp = W.fibre_pile(n_rods=24, n=20, L=0.2, per_row=2, rows=4, noise=1e-2, seed=W.SEED_BASE + 43)
    b = rod.RodBatch(inp, precision="f64")
    b.step(300)
    a, c = _both(b)
    # the contact potentials are summed in the order the grid's atomic binning
    # lists each bucket's nodes, which may differ between the two calls' contact
    # passes: equal to FP64 rounding of the sums
    assert np.allclose(a, c, rtol=1e-12, atol=1e-15 * np.abs(a).max())
    b.close()


def test_noalloc_energy_rejects_batches_beyond_its_buffer():
    from paper_2605_13766_amd import rod
    R = 262144 + 1
    print(f"case: {R} two-element rods, FP32 (rejected before any launch)", flush=True)
    b = rod.RodBatch(_vertical_rods(R), precision="f32", tile_waves=1, substeps=1)
    with pytest.raises(rod.RodError) as ei:
        b.energy_noalloc()
    assert ei.value.code == rod.ROD_EINVAL
    assert "262144" in str(ei.value)
    b.close()
    ok = rod.RodBatch(_vertical_rods(1000), precision="f32")
    ok.step(10)
    a, c = _both(ok)
    assert np.abs(a).max() > 0
    assert np.array_equal(a, c)
    ok.close()


def test_noalloc_energy_on_a_capsule_pile_with_a_stretched_rod():
    """Contact batches run a contact pass before the energies (the pairs'
    potentials) in both entry points; a rod flagged only as stretched
    (ROD_FLAG_STRETCHED) fails neither, and the two agree bit for bit."""
    from paper_2605_13766_amd import rod
    inp = W.fibre_pile(n_rods=24, n=8, L=0.248, per_row=2, rows=4, noise=1e-2, seed=68, contact=2)
    with rod.RodBatch(inp, precision="f64", substeps=1) as b:
        b.step(5)
        pos, vel, dr, om, t = b.get_state()
        a0 = inp.node_offset[2]
        n = inp.n_elems[2]
        pos[a0 + n] = pos[a0 + n - 1] + 1.4 * (pos[a0 + n] - pos[a0 + n - 1])
        b.set_state(pos, vel, dr, om, t)
        b.step(1)
        assert b.flags()[2] & rod.ROD_FLAG_STRETCHED
        a, c = _both(b)
        assert np.array_equal(a, c)
        assert a[:, 4].sum() > 0.0      # the contact potentials are in W_ext
