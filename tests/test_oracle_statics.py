"""Oracle pins: exact discrete equilibria and textbook statics.

Each configuration below is an equilibrium of the discrete model in closed
form, so the oracle's accelerations (Eq. 1a, 1b) must vanish to round-off:
rigid translation of a rest configuration, Hooke's axial stretch with the 1/e
of Eq. 1a, uniform torsion under an end couple, pure bending of a circular
polygon.  The damped cantilever reaches the Euler-Bernoulli deflection.
"""
import numpy as np
import pytest

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC


def _scale_acc(o):
    """Typical acceleration scale: accelerations after a small random perturbation."""
    rng = np.random.default_rng(0)
    p = ro.Oracle(o.inp)
    p.pos = p.pos + rng.normal(0, 1e-4, p.pos.shape) * o.rest_length.mean()
    p._mk()
    a, al = p.accel()
    return np.abs(a).max(), np.abs(al).max()


def test_rest_configuration_translated_is_force_free():
    inp = W.ragged_batch(n_rods=3, n_min=20, n_max=40, seed=7, damping=0.0)
    o = ro.Oracle(inp)
    _, kap, _ = o.strains()
    # declare the initial (curved) shape as the rest shape, then translate it
    moved = inp.copy()
    moved.rest_kappa = kap.copy()
    moved.rest_length = o.rest_length.copy()
    moved.position = inp.position + np.array([0.7, -1.3, 2.1])
    m = ro.Oracle(moved)
    a, al = m.accel()
    sa, sal = _scale_acc(m)
    assert np.abs(a).max() < 1e-9 * sa
    assert np.abs(al).max() < 1e-9 * sal


def test_hooke_axial_equilibrium():
    """Clamped rod, axial end force F: with n = Q^T S sigma / e the exact discrete
    equilibrium is e = EA / (EA - F), i.e. dL = F L / (EA - F)."""
    n, L, r, E, F = 20, 1.0, 0.01, 1e6, 2.0
    A, _ = RC.section(r)
    e = E * A / (E * A - F)
    nodes, Q = W.straight_rod(n, L)
    stretched = nodes * np.array([e, 1.0, 1.0])
    inp = RC.single(stretched, Q, E=E, radius=r, clamp0=1, rest_length=np.full(n, L / n),
                    end_force=[F, 0.0, 0.0])
    o = ro.Oracle(inp)
    a, al = o.accel()                      # node 0 / element 0 carry the clamp reaction
    assert np.abs(a[1:]).max() < 1e-8      # vs F/m_tip ~ 2/1.6e-2 ~ 1e2
    assert np.abs(al[1:]).max() < 1e-8
    # a damped run from the unstretched rod converges to dL = F L / (EA - F)
    inp2 = RC.single(nodes, Q, E=E, radius=r, clamp0=1, end_force=[F, 0.0, 0.0], damping=100.0,
                     dt=2e-5)
    o2 = ro.Oracle(inp2)
    o2.step(25000)
    dL = o2.pos[-1, 0] - L
    assert abs(dL / (F * L / (E * A - F)) - 1) < 1e-6
    assert abs(dL / (F * L / (E * A)) - 1) > 1e-6   # distinguishes the 1/e reading


def test_torsion_equilibrium():
    """End couple T about d3: uniform twist kappa3 = T / (G (I1 + I2)) is an exact
    discrete equilibrium; twist between first and last element T (L - lh) / B33."""
    n, L, r, E = 16, 0.5, 0.01, 1e6
    G = E / 1.5
    _, I = RC.section(r)
    B33 = G * 2 * I
    T = 1e-3
    k3 = T / B33
    nodes, Q = RC.twisted_rod(n, L, k3)
    lh = L / n
    couple = np.zeros((n, 3))
    couple[-1, 2] = T / lh            # couple per unit length on the last element
    o = ro.Oracle(RC.single(nodes, Q, E=E, radius=r, clamp0=1), elem_couple=couple)
    a, al = o.accel()
    assert np.abs(a[1:]).max() < 1e-10
    assert np.abs(al[1:]).max() < 1e-6 * (T * lh / (1000 * I * lh) * 1.0)
    psi_end = (n - 1) * lh * k3
    assert abs(psi_end - T * (L - lh) / B33) < 1e-14
    d1_last = Q[-1, 0]
    assert abs(np.arctan2(d1_last[2], d1_last[1]) - psi_end) < 1e-12


def test_pure_bending_equilibrium():
    """End couple M about d1: the polygonal arc with kappa1 = M / EI is an exact
    discrete equilibrium (kappa x B kappa = 0 for an isotropic section)."""
    n, ds, r, E = 24, 0.02, 0.01, 1e6
    _, I = RC.section(r)
    M = 2e-3
    phi = M / (E * I) * ds
    nodes, Q = RC.polygon_arc(n, ds, phi)
    couple = np.zeros((n, 3))
    couple[-1, 0] = M / ds
    o = ro.Oracle(RC.single(nodes, Q, E=E, radius=r, clamp0=1, rest_length=np.full(n, ds)),
                  elem_couple=couple)
    _, kap, _ = o.strains()
    assert np.abs(kap[:, 0] - M / (E * I)).max() < 1e-10
    a, al = o.accel()
    assert np.abs(a[1:]).max() < 1e-9
    assert np.abs(al[1:]).max() < 1e-4     # vs M ds/J ~ 5e3 without the couple


def test_bending_without_end_couple_is_not_equilibrium():
    n, ds, r, E = 24, 0.02, 0.01, 1e6
    _, I = RC.section(r)
    phi = 2e-3 / (E * I) * ds
    nodes, Q = RC.polygon_arc(n, ds, phi)
    o = ro.Oracle(RC.single(nodes, Q, E=E, radius=r, clamp0=1, rest_length=np.full(n, ds)))
    _, al = o.accel()
    assert np.abs(al[-1]).max() > 1e2


@pytest.mark.slow
def test_cantilever_static_euler_bernoulli():
    """Damped cantilever with tip force: deflection -> F L^3 / (3 EI) + F L / (alpha_c G A).

    The clamp holds element 0's director, so the beam is clamped at that element's
    midpoint: deflection at n elements follows L_eff = L - L/(2n), and the first-order
    Richardson extrapolation of n = 25, 50 recovers the continuum value."""
    E, r, L, F = 1e6, 0.01, 1.0, 1e-3
    A, I = RC.section(r)
    G = E / 1.5
    tips = {}
    for n in (25, 50):
        inp = W.single_cantilever(n=n, noise=0.0, dt=1e-4)
        inp.damping[:] = 1.1                 # ~ critical for the first mode (w1 = 0.556 rad/s)
        o = ro.Oracle(inp)
        o.step(int(round(20.0 / inp.dt)))
        tips[n] = -o.pos[-1, 2]
        Leff = L - L / (2 * n)
        ref = F * Leff ** 3 / (3 * E * I) + F * Leff / (4 / 3 * G * A)
        assert abs(tips[n] / ref - 1) < 0.01
    rich = 2 * tips[50] - tips[25]
    assert abs(rich / (F * L ** 3 / (3 * E * I) + F * L / (4 / 3 * G * A)) - 1) < 0.01


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("stretch", [1.0, 1.01])
def test_rotational_kinetic_energy_closed_form(axis, stretch):
    """T_rot of a straight rod whose elements all spin at w about one
    material axis, in closed form: 1/2 rho I_a L w^2 / e with I_1 = I_2 =
    pi r^4 / 4, I_3 = I_1 + I_2 (Eq. 1b's angular momentum density
    rho I omega / e); the rod stretched uniformly to e = 1.01 divides it by e."""
    n, L, r, rho, w = 20, 0.4, 0.01, 1000.0, 3.0
    nodes, Q = RC.twisted_rod(n, L, 0.0)
    om = np.zeros((n, 3))
    om[:, axis] = w
    inp = RC.single(nodes * stretch, Q, omega=om, radius=r, rho=rho, rest_length=np.full(n, L / n))
    e = ro.Oracle(inp).energy()[0]
    I1 = np.pi * r ** 4 / 4.0
    Ia = (I1, I1, 2.0 * I1)[axis]
    want = 0.5 * rho * Ia * L * w * w / stretch
    assert abs(e[1] / want - 1.0) < 1e-13
    assert e[0] == 0.0                      # nodes at rest
