"""Oracle pins: the rotation maps and the discrete strain measures.

The two maps are checked against an independent library (scipy's rotation
vectors); the strains against geometries whose curvature vector is known in
closed form from its definition kappa = ax(Q dQ^T/ds) (Methods, "Cosserat rod
dynamics"): a twisted straight rod, a polygonal arc and a helix carried by
its Frenet frame.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import rodoracle as ro
from paper_2605_13766_amd import workloads as W
import rodcases as RC


@pytest.mark.parametrize("scale", [0.0, 1e-12, 1e-7, 1e-3, 0.3, 1.5, 3.0])
def test_rodrigues_matches_scipy(scale):
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = rng.normal(size=3)
        u = u / np.linalg.norm(u) * scale
        E = ro.rodrigues(u)
        ref = Rotation.from_rotvec(u).as_matrix()
        assert np.abs(E - ref).max() < 1e-15 * 4
        assert np.abs(E @ E.T - np.eye(3)).max() < 1e-15 * 4


@pytest.mark.parametrize("scale", [1e-12, 1e-8, 1e-5, 1e-2, 0.5, 1.5, 2.5, 3.1])
def test_logmap_matches_scipy(scale):
    rng = np.random.default_rng(2)
    for _ in range(20):
        u = rng.normal(size=3)
        u = u / np.linalg.norm(u) * scale
        R = Rotation.from_rotvec(u).as_matrix()
        got = ro.logmap(R)
        ref = Rotation.from_matrix(R).as_rotvec()
        assert np.abs(got - ref).max() <= 1e-15 * 8 + 1e-13 * scale
        assert np.abs(got - u).max() <= 1e-15 * 8 + 1e-13 * scale


def test_logmap_inverts_rodrigues():
    rng = np.random.default_rng(3)
    for _ in range(200):
        u = rng.normal(size=3)
        u *= rng.uniform(0, 3.0) / np.linalg.norm(u)       # principal branch |u| < pi
        assert np.abs(ro.logmap(ro.rodrigues(u)) - u).max() < 1e-14


def _strains(nodes, Q, **kw):
    o = ro.Oracle(RC.single(nodes, Q, **kw))
    return o.strains()


def test_twist_curvature_closed_form():
    # psi' = 3 rad/m about d3: kappa = (0, 0, 3), sigma = 0, e = 1
    nodes, Q = RC.twisted_rod(20, 0.2, 3.0)
    sig, kap, dil = _strains(nodes, Q)
    assert np.abs(kap - np.array([0.0, 0.0, 3.0])).max() < 1e-12
    assert np.abs(sig).max() < 1e-14
    assert np.abs(dil - 1).max() < 1e-14


def test_arc_curvature_closed_form():
    # chord directions turning by phi about d1: kappa = (phi/ds, 0, 0) exactly
    ds, phi = 0.01, 0.03
    nodes, Q = RC.polygon_arc(30, ds, phi)
    sig, kap, _ = _strains(nodes, Q)
    assert np.abs(kap - np.array([phi / ds, 0.0, 0.0])).max() < 1e-11
    assert np.abs(sig).max() < 1e-13


def test_helix_curvature_frenet():
    # Frenet frame (N, B, T) of a helix rotates uniformly: Q_k Q_{k+1}^T = exp(ds [kappa]x)
    # exactly, so kappa = (0, curvature, torsion) to round-off once rest lengths are ds.
    ds = 0.01
    nodes, Q, kF, tF = RC.helix_frenet(40, ds, a=0.2, b=0.1)
    sig, kap, _ = _strains(nodes, Q, rest_length=np.full(40, ds))
    assert np.abs(kap - np.array([0.0, kF, tF])).max() < 1e-10 * max(kF, tF)


def test_strains_rigid_motion_invariant():
    """Strains are unchanged by r -> R r + c, Q -> Q R^T."""
    rng = np.random.default_rng(4)
    inp = W.ragged_batch(n_rods=3, n_min=20, n_max=40, seed=9)
    o = ro.Oracle(inp)
    s0, k0, e0 = o.strains()
    Rm = RC.random_rotation(rng)
    c = rng.normal(size=3)
    moved = inp.copy()
    moved.position = inp.position @ Rm.T + c
    moved.director = inp.director @ Rm.T
    moved.rest_length = o.rest_length.copy()
    s1, k1, e1 = ro.Oracle(moved).strains()
    assert np.abs(s1 - s0).max() < 1e-12
    assert np.abs(k1 - k0).max() < 1e-10 * max(1.0, np.abs(k0).max())
    assert np.abs(e1 - e0).max() < 1e-12     # |r| ~ 5 m, |dr| ~ 1e-2 m


def test_director_update_sign():
    """omega = ax(Q dQ^T/dt): a spinning rod's d1 turns about d3 by +w t (right hand)."""
    n, w = 8, 7.0
    nodes, Q = W.straight_rod(n, 0.08)
    om = np.tile([0.0, 0.0, w], (n, 1))
    o = ro.Oracle(RC.single(nodes, Q, omega=om, dt=1e-4))
    o.step(500)
    th = w * o.time
    d1 = np.array([0.0, np.cos(th), np.sin(th)])   # initial d1 = y, d3 = x
    assert np.abs(o.dir[:, 0, :] - d1).max() < 1e-12
    assert np.abs(o.pos - nodes).max() < 1e-15
    # the finite-difference definition ax(Q dQ^T)/dt recovers omega
    o2 = ro.Oracle(RC.single(nodes, Q, omega=np.tile([0.3, -0.2, 0.5], (n, 1)), E=1e-9, G=1e-9,
                             dt=1e-6))
    Qa = o2.dir.copy()
    o2.step(1)
    U = Qa[0] @ (o2.dir[0] - Qa[0]).T
    ax = 0.5 * np.array([U[2, 1] - U[1, 2], U[0, 2] - U[2, 0], U[1, 0] - U[0, 1]])
    assert np.abs(ax / 1e-6 - np.array([0.3, -0.2, 0.5])).max() < 1e-6
