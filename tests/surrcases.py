"""Shared set-up of the learned-coarse-step GPU tests: carpet rods at 64
elements whose start state comes from the FP64 oracle (never from the GPU),
loaded into an FP32 batch."""
import numpy as np

from paper_2605_13766_amd import workloads as W

N = 64
L = 0.01   # rod length of the carpet rods


def carpet(n_rods, seed_shift=0):
    return W.surrogate_at_scale(n_rods=n_rods, n=N, seed=W.SEED_BASE + 5 + seed_shift)


def oracle_run(inp, steps, state=None, t0=0.0):
    """FP64 oracle state after `steps` plain steps (from `state` at t0, or the
    initial state), and its time."""
    from oracle.rodoracle import Oracle
    o = Oracle(inp, t0=t0)
    if state is not None:
        o.pos[:], o.vel[:], o.dir[:], o.omega[:] = (np.asarray(a, float).reshape(b.shape)
                                                    for a, b in zip(state, (o.pos, o.vel, o.dir, o.omega)))
    if steps:
        o.step(steps)
    return o.state(), o.time


def gpu_batch(inp, state=None, t=0.0):
    from paper_2605_13766_amd import rod
    b = rod.RodBatch(inp, precision="f32")
    if state is not None:
        b.set_state(*state, t=t)
    return b


def gpu_state(b):
    p, v, d, w, t = b.get_state()
    return (p, v, d, w), t


def pos_err(ref, b):
    """Per rod max_j |r_j - r_j(ref)| / L of two batches (or a batch and a
    state tuple)."""
    p1 = (ref[0] if isinstance(ref, tuple) else ref.get_state()[0]).reshape(-1, N + 1, 3)
    p2 = b.get_state()[0].reshape(-1, N + 1, 3)
    return np.linalg.norm(p2 - p1, axis=2).max(axis=1) / L
