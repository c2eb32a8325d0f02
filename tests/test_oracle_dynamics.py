"""Oracle pins: invariants and closed forms of the time-stepped dynamics.

* orthonormality of the directors under the exponential-map update;
* linear momentum: the difference operator telescopes, so free rods conserve
  sum m v exactly, and linear damping scales it by (1 - gamma h) per step;
* angular momentum of a free rod (orbital + spin, spin density rho I omega / e,
  Eq. 1b) is conserved up to time-discretisation error;
* rigid-motion covariance of whole trajectories;
* energy without damping bounded, no drift;
* Euler's torque-free equations for a spinning element (the
  (rho I omega / e) x omega term), conservation of rho I omega / e under axial
  stretching (the (rho I omega / e^2) de/dt term);
* Euler-Bernoulli cantilever under a suddenly applied tip force, by modal
  superposition.

The mutation test removes each couple term from the oracle in turn and checks
that some pin here fails, so none of them is vacuous.
"""
import numpy as np
import pytest

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC


# --------------------------------------------------------------- helpers

def lumped_masses(o):
    out = []
    eo = 0
    for r in range(o.R):
        n = o.n_elems[r]
        A, _ = RC.section(o.inp.radius[r])
        lh = o.rest_length[eo:eo + n]
        m = np.zeros(n + 1)
        m[:-1] += 0.5 * o.inp.density[r] * A * lh
        m[1:] += 0.5 * o.inp.density[r] * A * lh
        out.append(m)
        eo += n
    return np.concatenate(out)


def angular_momentum(o):
    """sum_j m_j r_j x v_j + sum_i Q_i^T (J_i omega_i / e_i), J_i = rho I lh_i."""
    m = lumped_masses(o)
    L = np.sum(m[:, None] * np.cross(o.pos, o.vel), axis=0)
    _, _, dil = o.strains()
    eo = 0
    for r in range(o.R):
        n = o.n_elems[r]
        _, I = RC.section(o.inp.radius[r])
        lh = o.rest_length[eo:eo + n]
        J = o.inp.density[r] * I * np.stack([lh, lh, 2 * lh], axis=1)
        h = J * o.omega[eo:eo + n] / dil[eo:eo + n, None]
        L += np.einsum("iba,ib->a", o.dir[eo:eo + n], h)
        eo += n
    return L


def free_tumbling_rod(seed=11):
    rng = np.random.default_rng(5)
    inp = W.ragged_batch(n_rods=1, n_min=40, n_max=40, damping=0.0, seed=seed)
    inp.velocity = rng.normal(0, 0.05, size=inp.velocity.shape)
    inp.omega = rng.normal(0, 2.0, size=inp.omega.shape)
    return inp


# --------------------------------------------------------------- pins as (value, tolerance)

def pin_angular_momentum(drop=0):
    o = ro.Oracle(free_tumbling_rod(), drop_term=drop)
    L0 = angular_momentum(o)
    o.step(2000)
    return np.linalg.norm(angular_momentum(o) - L0) / np.linalg.norm(L0), 1e-6


def pin_precession(drop=0, dt=1e-4, steps=1000):
    """Torque-free symmetric element, J3 = 2 J1: (w1, w2) turns at rate w3."""
    n = 10
    nodes, Q = W.straight_rod(n, 0.1)
    w3, wp = 10.0, 1.0
    inp = RC.single(nodes, Q, E=1e-6, G=1e-6, dt=dt, omega=np.tile([wp, 0.0, w3], (n, 1)))
    o = ro.Oracle(inp, drop_term=drop)
    o.step(steps)
    t = o.time
    ref = np.array([wp * np.cos(w3 * t), wp * np.sin(w3 * t), w3])
    return np.abs(o.omega - ref).max(), 1e-3


def pin_dilatation(drop=0):
    """rho I omega / e is conserved when only the dilatation term acts:
    spin about d3, axial vibration, negligible shear modulus."""
    n = 20
    nodes, Q = W.straight_rod(n, 0.2)
    vel = np.zeros((n + 1, 3))
    vel[:, 0] = 0.05 * (np.arange(n + 1) / n - 0.5)
    inp = RC.single(nodes, Q, E=1e6, G=1e-3, dt=1e-5, vel=vel,
                    omega=np.tile([0.0, 0.0, 10.0], (n, 1)))
    o = ro.Oracle(inp, drop_term=drop)
    _, _, e0 = o.strains()
    r0 = o.omega[:, 2] / e0
    worst, emax = 0.0, 0.0
    for _ in range(20):
        o.step(100)
        _, _, e = o.strains()
        worst = max(worst, np.abs(o.omega[:, 2] / e / r0 - 1).max())
        emax = max(emax, np.abs(e - 1).max())
    assert emax > 3e-4          # the rod really stretches
    return worst, 2e-5


def pin_bending_arc(drop=0):
    """Pure-bending polygon with end couple: residual angular acceleration."""
    n, ds, r, E = 24, 0.02, 0.01, 1e6
    _, I = RC.section(r)
    M = 2e-3
    nodes, Q = RC.polygon_arc(n, ds, M / (E * I) * ds)
    couple = np.zeros((n, 3))
    couple[-1, 0] = M / ds
    o = ro.Oracle(RC.single(nodes, Q, E=E, radius=r, clamp0=1, rest_length=np.full(n, ds)),
                  elem_couple=couple, drop_term=drop)
    _, al = o.accel()
    return np.abs(al[1:]).max(), 1e-4


def pin_cantilever_transient(drop=0):
    inp = W.single_cantilever(noise=0.0)
    o = ro.Oracle(inp, drop_term=drop)
    A, I = RC.section(0.01)
    worst = 0.0
    for T in (5000, 10000):
        o.step(T - o.step_index)
        ref = RC.cantilever_modal_tip(o.time, 1e-3, 1e6, I, 1000.0, A, 1.0)
        worst = max(worst, abs(-o.pos[-1, 2] / ref - 1))
    return worst, 0.01


ALL_PINS = [pin_angular_momentum, pin_precession, pin_dilatation, pin_bending_arc,
            pin_cantilever_transient]


# --------------------------------------------------------------- tests

@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda f: f.__name__)
def test_pin_holds(pin):
    val, tol = pin()
    assert val < tol, (pin.__name__, val, tol)


def test_precession_first_order_in_h():
    """The explicit gyroscopic kick is first order: halving h halves the error."""
    e1, _ = pin_precession(dt=2e-4, steps=500)
    e2, _ = pin_precession(dt=1e-4, steps=1000)
    assert 1.7 < e1 / e2 < 2.3


@pytest.mark.parametrize("drop", [1, 2, 3, 4, 5])
def test_each_couple_term_is_pinned(drop):
    """Removing any one couple term of Eq. 1b from the oracle breaks some pin:
    1 d/ds(B kappa/e^3), 2 kappa x B kappa/e^3, 3 Q t x S sigma,
    4 (rho I omega/e) x omega, 5 (rho I omega/e^2) de/dt."""
    failed = []
    for pin in ALL_PINS:
        val, tol = pin(drop)
        if not val < tol:
            failed.append(pin.__name__)
    assert failed, f"dropping term {drop} went unnoticed"


def test_orthonormality_preserved():
    inp = W.single_cantilever()
    o = ro.Oracle(inp)
    o.step(10000)
    QQt = np.einsum("iab,icb->iac", o.dir, o.dir)
    assert np.abs(QQt - np.eye(3)).max() < 1e-12
    assert np.all(np.linalg.det(o.dir) > 0)


def test_linear_momentum_free_rods():
    inp = W.ragged_batch(n_rods=4, n_min=16, n_max=40, damping=0.0, seed=3)
    rng = np.random.default_rng(8)
    inp.velocity = rng.normal(0, 0.02, size=inp.velocity.shape)
    inp.omega = rng.normal(0, 1.0, size=inp.omega.shape)
    o = ro.Oracle(inp)
    m = lumped_masses(o)
    P0 = [np.sum(m[no:no + n + 1, None] * o.vel[no:no + n + 1], axis=0)
          for no, n in zip(inp.node_offset, inp.n_elems)]
    o.step(1000)
    for k, (no, n) in enumerate(zip(inp.node_offset, inp.n_elems)):
        P1 = np.sum(m[no:no + n + 1, None] * o.vel[no:no + n + 1], axis=0)
        scale = np.sum(m[no:no + n + 1]) * 0.02
        assert np.abs(P1 - P0[k]).max() < 1e-12 * scale


def test_linear_damping_scales_momentum():
    gamma, N = 0.1, 1000
    inp = W.ragged_batch(n_rods=2, n_min=16, n_max=40, damping=gamma, seed=4)
    rng = np.random.default_rng(9)
    inp.velocity = rng.normal(0, 0.02, size=inp.velocity.shape)
    o = ro.Oracle(inp)
    m = lumped_masses(o)
    P0 = np.sum(m[:, None] * o.vel, axis=0)
    o.step(N)
    P1 = np.sum(m[:, None] * o.vel, axis=0)
    fac = (1 - gamma * inp.dt) ** N
    assert np.abs(P1 - fac * P0).max() < 1e-12 * np.abs(P0).max()


def test_rigid_translation_damping_closed_form():
    gamma, N, v0 = 0.1, 2000, np.array([0.3, -0.2, 0.1])
    n = 12
    nodes, Q = W.straight_rod(n, 0.12)
    inp = RC.single(nodes, Q, damping=gamma, vel=np.tile(v0, (n + 1, 1)), dt=1e-5)
    o = ro.Oracle(inp)
    o.step(N)
    fac = (1 - gamma * inp.dt) ** N
    assert np.abs(o.vel - fac * v0).max() < 1e-11     # round-off strains of the moving rod
    assert np.abs(o.dir - Q).max() < 1e-13


def test_trajectory_rigid_rotation_covariant():
    rng = np.random.default_rng(6)
    inp = W.ragged_batch(n_rods=2, n_min=20, n_max=30, damping=0.0, seed=5)
    inp.velocity = rng.normal(0, 0.02, size=inp.velocity.shape)
    inp.omega = rng.normal(0, 1.0, size=inp.omega.shape)
    o = ro.Oracle(inp)
    Rm = RC.random_rotation(rng)
    moved = inp.copy()
    moved.position = inp.position @ Rm.T
    moved.velocity = inp.velocity @ Rm.T
    moved.director = inp.director @ Rm.T
    moved.rest_length = o.rest_length.copy()
    m = ro.Oracle(moved)
    o.step(1000)
    m.step(1000)
    L = 0.01 * inp.n_elems.max()
    assert np.abs(m.pos - o.pos @ Rm.T).max() < 1e-12 * max(L, np.abs(o.pos).max())
    # round-off of the rotated copy grows through the (stiff) dynamics; 1e-10 is far
    # below any physical effect of a wrong frame convention (O(1))
    assert np.abs(m.dir - o.dir @ Rm.T).max() < 1e-10
    assert np.abs(m.omega - o.omega).max() < 1e-8 * max(1.0, np.abs(o.omega).max())


def test_energy_conserved_without_damping():
    """Cantilever as configured (undamped, tip force): H = T + U + W_ext stays within
    1e-4 of max(T+U) and the deviation shrinks when h is halved."""
    devs = []
    for dt in (2e-5, 1e-5):
        inp = W.single_cantilever(dt=dt)
        o = ro.Oracle(inp)
        H0 = o.energy()[0].sum()
        worst, tu = 0.0, 0.0
        steps = int(round(0.1 / dt))
        for _ in range(10):
            o.step(steps // 10)
            e = o.energy()[0]
            worst = max(worst, abs(e.sum() - H0))
            tu = max(tu, e[:4].sum())
        assert worst < 1e-4 * tu
        devs.append(worst)
    assert devs[1] < devs[0]


def test_energy_terms_closed_form():
    """U_bend of the pure-bending polygon = 1/2 EI kappa^2 (n-1) ds; U_shear of the
    Hooke state = 1/2 EA (e-1)^2 L; T_lin of a rigid translation = 1/2 M v^2."""
    n, ds, r, E = 24, 0.02, 0.01, 1e6
    A, I = RC.section(r)
    k1 = 0.5
    nodes, Q = RC.polygon_arc(n, ds, k1 * ds)
    o = ro.Oracle(RC.single(nodes, Q, E=E, radius=r, rest_length=np.full(n, ds)))
    e = o.energy()[0]
    assert abs(e[3] / (0.5 * E * I * k1 ** 2 * (n - 1) * ds) - 1) < 1e-10
    assert abs(e[2]) < 1e-20
    ex = 1.001
    nodes, Q = W.straight_rod(n, n * ds)
    o = ro.Oracle(RC.single(nodes * np.array([ex, 1, 1]), Q, E=E, radius=r,
                            rest_length=np.full(n, ds), vel=np.tile([0.0, 0.2, 0.0], (n + 1, 1))))
    e = o.energy()[0]
    assert abs(e[2] / (0.5 * E * A * (ex - 1) ** 2 * n * ds) - 1) < 1e-9
    assert abs(e[0] / (0.5 * 1000.0 * A * n * ds * 0.04) - 1) < 1e-12
