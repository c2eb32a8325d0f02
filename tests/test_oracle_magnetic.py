"""Pins of the oracle's magnetic couple (Methods, "Magnetized filaments",
Eq. 2: c_mag = m x (Q b(t)) per unit length, m in the material frame, b the
homogeneous lab field) against rigid-body physics of a stiff magnetized rod:

* sign: a damped rod whose axial magnetization starts perpendicular to a
  static field turns to point along +b (a dipole's torque m x B turns m
  toward B), not along -b;
* time dependence: in a slowly rotating field b(t) = B0 (cos wt, sin wt, 0)
  the damped rod follows the field, pointing along +y a quarter period later;
* magnitude: released at a small angle from a static field, the rod swings
  about it as a compass needle, omega^2 = m_tot B0 / I with m_tot = |m| L and
  I the rod's moment of inertia about its centre (lumped node masses plus the
  elements' own rotational inertia); the period within 1%.
"""
import numpy as np

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC

N, L, RAD, RHO, E = 10, 0.1, 0.005, 1000.0, 1e9
M0, B0 = 2.6e3, 0.01        # A m per unit length, tesla


def _rod(axis, damping, dt, field, field_freq=0.0):
    nodes, Q = W.straight_rod(N, L, direction=axis, d1=(0, 1, 0) if abs(axis[1]) < 0.5 else (0, 0, 1))
    inp = RC.single(nodes, Q, E=E, radius=RAD, rho=RHO, damping=damping, dt=dt)
    inp.magnetization = np.tile([0.0, 0.0, M0], (N, 1))     # along d3
    inp.field = np.asarray(field, float)
    inp.field_freq = field_freq
    return inp


def _axis(o):
    d = o.pos[-1] - o.pos[0]
    return d / np.linalg.norm(d)


def test_static_field_aligns_the_magnetization():
    inp = _rod((0, 0, 1), damping=600.0, dt=1e-6, field=[B0, 0, 0, 0, 0, 0, 0, 0, 0])
    o = ro.Oracle(inp)
    o.step(50000)
    a = _axis(o)
    print("axis after 0.05 s", a)
    assert a[0] > 0.99


def test_rotating_field_is_followed():
    f = 5.0
    inp = _rod((1, 0, 0), damping=600.0, dt=1e-6, field=[0, 0, 0, B0, 0, 0, 0, B0, 0], field_freq=f)
    o = ro.Oracle(inp)
    o.step(int(round(0.25 / f / 1e-6)))
    a = _axis(o)
    print("axis a quarter field period later", a)
    assert a[1] > 0.99 and abs(a[0]) < 0.1


def test_compass_needle_period():
    th0 = 0.05
    inp = _rod((0, 0, 1), damping=0.0, dt=1e-6, field=[B0 * np.sin(th0), 0, B0 * np.cos(th0), 0, 0, 0, 0, 0, 0])
    A, I1 = RC.section(RAD)
    ds = L / N
    s = np.arange(N + 1) * ds
    m = np.full(N + 1, RHO * A * ds)
    m[0] = m[-1] = 0.5 * RHO * A * ds
    I = np.sum(m * (s - L / 2) ** 2) + N * RHO * I1 * ds
    T = 2 * np.pi / np.sqrt(M0 * L * B0 / I)
    o = ro.Oracle(inp)
    dt = inp.dt
    ts, th = [], []
    for k in range(int(1.3 * T / dt) // 50):
        o.step(50)
        a = _axis(o)
        ts.append(o.time)
        th.append(np.arctan2(a[0], a[2]) - th0)
    th = np.array(th)
    ts = np.array(ts)
    # upward zero crossings of the angle from the field: one period apart
    up = [ts[i] - th[i] * (ts[i + 1] - ts[i]) / (th[i + 1] - th[i])
          for i in range(len(th) - 1) if th[i] < 0 <= th[i + 1]]
    print("expected period", T, "crossings", up)
    assert len(up) >= 1
    down = [ts[i] - th[i] * (ts[i + 1] - ts[i]) / (th[i + 1] - th[i])
            for i in range(len(th) - 1) if th[i] > 0 >= th[i + 1]]
    period = 2 * abs(up[0] - down[0]) if down else None
    print("measured half-period crossing gap -> period", period)
    assert period is not None and abs(period / T - 1) < 0.01
