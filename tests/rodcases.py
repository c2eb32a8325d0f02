"""Hand-built rod configurations with known answers (tests only).

Each builder returns a ``RodInputs`` batch plus whatever closed-form quantity
the test compares against.  Geometry is written out directly from its
definition (straight rods, twisted rods, polygonal arcs, helices with their
Frenet frames) and does not use the oracle.
"""
from __future__ import annotations

import numpy as np

from paper_2605_13766_amd import workloads as W


def section(radius):
    A = np.pi * radius ** 2
    I = np.pi * radius ** 4 / 4.0
    return A, I


def single(nodes, Q, *, E=1e6, G=None, radius=0.01, rho=1000.0, alpha_c=4.0 / 3.0,
           damping=0.0, clamp0=0, clamp1=0, dt=1e-5, vel=None, omega=None, rest_length=None,
           rest_kappa=None, end_force=None):
    G = E / 1.5 if G is None else G
    n = Q.shape[0]
    return W.RodInputs(
        n_elems=np.array([n], np.int32), position=np.ascontiguousarray(nodes, float),
        velocity=np.zeros_like(nodes) if vel is None else np.ascontiguousarray(vel, float),
        director=np.ascontiguousarray(Q, float),
        omega=np.zeros((n, 3)) if omega is None else np.ascontiguousarray(omega, float),
        density=np.array([rho]), youngs=np.array([E]), shear_modulus=np.array([G]),
        radius=np.array([radius]), shear_coeff=np.array([alpha_c]), damping=np.array([damping]),
        bc_start=np.array([clamp0], np.int32), bc_end=np.array([clamp1], np.int32), dt=dt,
        rest_length=rest_length, rest_kappa=rest_kappa,
        end_force=None if end_force is None else np.asarray(end_force, float).reshape(1, 3))


def twisted_rod(n, L, psi_rate):
    """Straight rod along x whose frame turns about d3 = x at psi' = psi_rate.

    Element i has d1 = cos(psi_i) y + sin(psi_i) z, d2 = -sin(psi_i) y + cos(psi_i) z,
    psi_i = i * (L/n) * psi_rate.  Its curvature vector is (0, 0, psi_rate).
    """
    ds = L / n
    nodes = np.stack([np.linspace(0, L, n + 1), np.zeros(n + 1), np.zeros(n + 1)], axis=1)
    Q = np.zeros((n, 3, 3))
    for i in range(n):
        p = i * ds * psi_rate
        Q[i, 0] = [0.0, np.cos(p), np.sin(p)]
        Q[i, 1] = [0.0, -np.sin(p), np.cos(p)]
        Q[i, 2] = [1.0, 0.0, 0.0]
    return nodes, Q


def polygon_arc(n, ds, phi):
    """Planar polygon of n chords of length ds, each turned by phi from the previous.

    d1 = z (binormal), d3_i = (cos a_i, sin a_i, 0) with a_i = i*phi, d2 = d3 x d1.
    Its discrete curvature is (phi/ds, 0, 0) exactly.
    """
    Q = np.zeros((n, 3, 3))
    nodes = np.zeros((n + 1, 3))
    for i in range(n):
        a = i * phi
        d3 = np.array([np.cos(a), np.sin(a), 0.0])
        d1 = np.array([0.0, 0.0, 1.0])
        Q[i] = [d1, np.cross(d3, d1), d3]
        nodes[i + 1] = nodes[i] + ds * d3
    return nodes, Q


def helix_frenet(n, ds, a, b):
    """Helix r(s) = (a cos(s/c), a sin(s/c), b s/c), c = sqrt(a^2 + b^2), with rows
    (N, B, T) of its Frenet frame at the element midpoints.

    Curvature a/c^2, torsion b/c^2; the material curvature vector of this frame
    is (0, a/c^2, b/c^2).
    """
    c = np.hypot(a, b)
    s = np.arange(n + 1) * ds
    nodes = np.stack([a * np.cos(s / c), a * np.sin(s / c), b * s / c], axis=1)
    Q = np.zeros((n, 3, 3))
    for i in range(n):
        sm = (i + 0.5) * ds
        T = np.array([-a * np.sin(sm / c), a * np.cos(sm / c), b]) / c
        N = np.array([-np.cos(sm / c), -np.sin(sm / c), 0.0])
        B = np.cross(T, N)
        Q[i] = [N, B, T]
    return nodes, Q, a / c ** 2, b / c ** 2


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def cantilever_modal_tip(t, F, E, I, rho, A, L, n_modes=400):
    """Tip deflection of an Euler-Bernoulli cantilever under a suddenly applied tip
    force F, by modal superposition: sum_n 4F/(rho A L w_n^2) (1 - cos w_n t),
    w_n = (beta_n L)^2 sqrt(EI/(rho A L^4)), cos(b) cosh(b) = -1."""
    from scipy.optimize import brentq
    g = lambda x: np.cos(x) + 1.0 / np.cosh(x)
    roots = []
    for k in range(n_modes):
        c0 = (k + 0.5) * np.pi
        if k < 12:
            roots.append(brentq(g, max(c0 - 1.4, 0.1), c0 + 1.4))
        else:
            roots.append(c0)
    bl = np.array(roots)
    om = bl ** 2 * np.sqrt(E * I / (rho * A * L ** 4))
    return float(np.sum(4.0 * F / (rho * A * L * om ** 2) * (1.0 - np.cos(om * t))))
