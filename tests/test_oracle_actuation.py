"""Pins of the oracle's gravity and muscle torques (Results, "Active matter":
the filaments settle under gravity, then are driven by internal, net-zero
muscular torques prescribed as a travelling wave).

Gravity (nodal force m_j g):
* a free rod falls with its centre of mass on the closed-form parabola and
  its shape unchanged (internal forces cancel; position Verlet is exact for a
  constant acceleration);
* a damped cantilever under its own weight settles at the Euler-Bernoulli
  deflection q L^4 / (8 E I) plus the shear term q L^2 / (2 alpha_c G A), with
  the clamp at element 0's midpoint (L_eff = L - L / (2n), as for the
  tip-force cantilever);
* without damping T + U + W_ext (W_ext holding the work of gravity) stays
  constant while the cantilever swings.

Muscle torques (active moment beta sin(2 pi f t - q s_k + phi) axis added to
the internal moment at Voronoi point k):
* a static moment about d1 on a rod with rest curvature about d2 settles at
  kappa = kappa0 - m / B component by component, which holds only when the
  moment is part of the internal moment (it then also enters kappa x M);
* a slow travelling wave is followed quasi-statically: kappa_1 at the
  Voronoi points tracks -beta sin(2 pi f t - q s_k + phi) / (E I) within the
  lag of the damped response, while a wave running the other way, or s_k
  taken at the element midpoints instead, misses by several times that.
"""
import numpy as np

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC


def _masses(n, L, rad, rho=1000.0):
    A, _ = RC.section(rad)
    m = np.full(n + 1, rho * A * L / n)
    m[0] = m[-1] = 0.5 * rho * A * L / n
    return m


def test_free_fall_is_a_parabola():
    n, L, rad = 20, 0.2, 0.005
    nodes, Q = W.straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0))
    v0 = np.array([0.1, 0.0, 0.3])
    inp = RC.single(nodes, Q, E=1e6, radius=rad, dt=1e-5, vel=np.tile(v0, (n + 1, 1)))
    inp.gravity = np.array([0.0, -1.0, -9.81])
    o = ro.Oracle(inp)
    o.step(3000)
    t = o.time
    m = _masses(n, L, rad)
    com = (m[:, None] * o.pos).sum(0) / m.sum()
    com0 = (m[:, None] * nodes).sum(0) / m.sum()
    assert np.abs(com - (com0 + v0 * t + 0.5 * inp.gravity * t * t)).max() < 1e-12
    assert np.abs((o.pos - com) - (nodes - com0)).max() < 1e-12


def test_cantilever_settles_under_its_own_weight():
    n, L, rad, E = 50, 0.5, 0.01, 1e9
    nodes, Q = W.straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0))
    inp = RC.single(nodes, Q, E=E, radius=rad, dt=4e-6, damping=100.0, clamp0=1)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    A, I = RC.section(rad)
    q = 1000.0 * A * 9.81
    Le = L - L / (2 * n)
    ref = q * Le ** 4 / (8 * E * I) + q * Le ** 2 / (2 * (4 / 3) * (E / 1.5) * A)
    o = ro.Oracle(inp)
    o.step(80000)
    tip = -o.pos[-1, 2]
    print("tip", tip, "Euler-Bernoulli + shear", ref)
    assert abs(tip / ref - 1) < 5e-3


def test_energy_with_gravity_is_conserved():
    n, L, rad, E = 50, 0.5, 0.01, 1e9
    nodes, Q = W.straight_rod(n, L, direction=(1, 0, 0), d1=(0, 1, 0))
    inp = RC.single(nodes, Q, E=E, radius=rad, dt=4e-6, clamp0=1)
    inp.gravity = np.array([0.0, 0.0, -9.81])
    o = ro.Oracle(inp)
    H0 = o.energy().sum()
    H, swing = [], []
    for _ in range(20):
        o.step(2500)
        e = o.energy()
        H.append(e.sum())
        swing.append(e[0, :4].sum())
    drift = np.abs(np.array(H) - H0).max()
    print("energy drift", drift, "largest T + U", max(swing))
    assert drift < 1e-6 * max(swing)


def _muscle(inp, beta, axis, f, q, phi):
    n = int(inp.n_elems[0])
    inp.muscle_amp = np.full(n - 1, float(beta))
    inp.muscle_axis = np.array([axis], float)
    inp.muscle_freq = np.array([f], float)
    inp.muscle_wavenumber = np.array([q], float)
    inp.muscle_phase = np.array([phi], float)
    return inp


def test_static_muscle_moment_joins_the_internal_moment():
    n, L, rad, E = 40, 0.2, 0.005, 1e7
    nodes, Q = W.straight_rod(n, L, direction=(0, 0, 1), d1=(1, 0, 0))
    _, I = RC.section(rad)
    B1 = E * I
    beta, k0y = 1.5 * B1, 2.0
    inp = RC.single(nodes, Q, E=E, radius=rad, damping=200.0, dt=2e-6,
                    rest_kappa=np.tile([0.0, k0y, 0.0], (n - 1, 1)))
    o = ro.Oracle(_muscle(inp, beta, (1.0, 0.0, 0.0), 0.0, 0.0, np.pi / 2))
    o.step(120000)
    _, kap, _ = o.strains()
    print("kappa", kap[[0, n // 2, -1]])
    assert np.abs(kap - [-beta / B1, k0y, 0.0]).max() < 1e-5 * k0y


def test_travelling_wave_is_followed():
    n, L, rad, E = 40, 0.2, 0.005, 1e7
    nodes, Q = W.straight_rod(n, L, direction=(0, 0, 1), d1=(1, 0, 0))
    _, I = RC.section(rad)
    B1 = E * I
    beta, f, q, phi = 1.5 * B1, 0.5, 2 * np.pi / L, 0.4
    inp = RC.single(nodes, Q, E=E, radius=rad, damping=200.0, dt=2e-6)
    o = ro.Oracle(_muscle(inp, beta, (1.0, 0.0, 0.0), f, q, phi))
    sk = np.arange(1, n) * (L / n)          # rest arc length of Voronoi point k
    amp = beta / B1
    for _ in range(4):
        o.step(25000)
        _, kap, _ = o.strains()
        t = o.time
        err = np.abs(kap[:, 0] + amp * np.sin(2 * np.pi * f * t - q * sk + phi)).max() / amp
        back = np.abs(kap[:, 0] + amp * np.sin(2 * np.pi * f * t + q * sk + phi)).max() / amp
        mid = np.abs(kap[:, 0] + amp * np.sin(2 * np.pi * f * t - q * (sk - L / (2 * n)) + phi)).max() / amp
        print(f"t {t:.3f}: error {err:.4f}, backward wave {back:.3f}, midpoint arc length {mid:.3f}")
        assert err < 0.04 and back > 0.5 and mid > 0.08
        assert np.abs(kap[:, 1:]).max() < 1e-9 * amp
