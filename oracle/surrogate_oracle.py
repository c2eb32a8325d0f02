"""FP64 CPU oracle of the learned coarse step's data path: window features,
training targets, applying predicted deltas, and the judge's error measures.

TEST INFRASTRUCTURE ONLY (tests, smoke, CPU baseline).  Definitions (the
library's own; the paper has no surrogate): for a rod with n elements there are
n + 1 windows; window w < n is centred on element c = w and targets node c and
element c, window n is centred on element n - 1 and targets node n (its
element outputs are masked).  tau = k * dt is the coarse step; lh_c is the
centre element's rest length; everything is expressed in the centre
element's director frame Q_c (rows d1, d2, d3).

Per stencil slot j = c + s, s = -2..2 (16 values, zero when j is outside the
rod): Q_c (x_j - x_c) / lh_c with x the element midpoint; Q_c (u_j - u_c) tau / lh_c
with u the element's mean node velocity; rows 0 and 1 of Q_j Q_c^T; omega_j tau;
a 1 flag.  Globals (16): Q_c v_p tau / lh_c and Q_c (r_p - x_c) / lh_c for the
target node p; log10(E / 1e6); radius / lh_c; log10(tau / T_b) with
T_b = lh_c^2 sqrt(rho A / (E I)); alpha_c; clamped-base flag; c / n; end flag;
couple amplitude (material x) / 1e-5 N m/m; sin and cos of the couple phase
2 pi f t + phi.

Targets (12) are the departures from free flight over tau (constant node
velocity, constant element angular velocity), which the apply step adds back:
Q_c (r_p(t+tau) - r_p(t) - v_p(t) tau) / lh_c; Q_c (v_p(t+tau) - v_p(t)) tau / lh_c;
theta - omega_c(t) tau with theta = log(Q_c(t) Q_c(t+tau)^T) (so
Q_c(t+tau) = exp(-[theta]x) Q_c(t)); (omega_c(t+tau) - omega_c(t)) tau.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 96
N_OUT = 12
AMP_SCALE = 1e-5


def _logvec(R):
    """Rotation vector of rotation matrices R [..., 3, 3] (atan2 form)."""
    w = 0.5 * np.stack([R[..., 2, 1] - R[..., 1, 2], R[..., 0, 2] - R[..., 2, 0], R[..., 1, 0] - R[..., 0, 1]], -1)
    s = np.linalg.norm(w, axis=-1)
    c = 0.5 * (np.trace(R, axis1=-2, axis2=-1) - 1.0)
    th = np.arctan2(s, c)
    f = np.where(s > 1e-12, th / np.where(s > 1e-12, s, 1.0), 1.0 + s * s / 6.0)
    return f[..., None] * w


def _expmap(u):
    """exp([u]x) for rotation vectors u [..., 3] (Rodrigues)."""
    th = np.linalg.norm(u, axis=-1)
    k = u / np.where(th > 0, th, 1.0)[..., None]
    K = np.zeros(u.shape[:-1] + (3, 3))
    K[..., 0, 1], K[..., 0, 2] = -k[..., 2], k[..., 1]
    K[..., 1, 0], K[..., 1, 2] = k[..., 2], -k[..., 0]
    K[..., 2, 0], K[..., 2, 1] = -k[..., 1], k[..., 0]
    s = np.sin(th)[..., None, None]
    c1 = (1.0 - np.cos(th))[..., None, None]
    return np.eye(3) + s * K + c1 * (K @ K)


def _nearest_rotation(A):
    """Orthogonal polar factor U V^T of A = U S V^T: the rotation closest to A
    in the Frobenius norm (A near a rotation, so det > 0)."""
    U, _, Vt = np.linalg.svd(A)
    return U @ Vt


def rod_views(inp):
    """Per-rod slices (node slice, element slice) of a RodInputs-like batch."""
    no, eo = inp.node_offset, inp.elem_offset
    return [(slice(no[r], no[r] + n + 1), slice(eo[r], eo[r] + n)) for r, n in enumerate(inp.n_elems)]


def window_features(inp, state, t, k):
    """Raw FP64 features [sum(n+1), 96] of every window of every rod."""
    pos, vel, Q, om = state
    tau = k * inp.dt
    out = []
    lh_all = (inp.rest_length if inp.rest_length is not None
              else np.concatenate([np.linalg.norm(np.diff(inp.position[ns], axis=0), axis=1)
                                   for ns, _ in rod_views(inp)]))
    for r, (ns, es) in enumerate(rod_views(inp)):
        n = int(inp.n_elems[r])
        x = pos[ns]
        v = vel[ns]
        q = Q[es]
        w = om[es]
        lh = lh_all[es]
        mid = 0.5 * (x[:-1] + x[1:])
        u = 0.5 * (v[:-1] + v[1:])
        A = np.pi * inp.radius[r] ** 2
        I = np.pi * inp.radius[r] ** 4 / 4.0
        amp = 0.0 if inp.couple_amp is None else inp.couple_amp[r][0]
        f = 0.0 if inp.couple_freq is None else inp.couple_freq[r]
        ph = 0.0 if inp.couple_phase is None else inp.couple_phase[r]
        phase = 2.0 * np.pi * f * t + ph
        F = np.zeros((n + 1, N_FEAT))
        for wi in range(n + 1):
            c = min(wi, n - 1)
            p = wi if wi < n else n
            Qc = q[c]
            L = lh[c]
            for si, s in enumerate(range(-2, 3)):
                j = c + s
                if j < 0 or j >= n:
                    continue
                o = 16 * si
                F[wi, o:o + 3] = Qc @ (mid[j] - mid[c]) / L
                F[wi, o + 3:o + 6] = Qc @ (u[j] - u[c]) * tau / L
                Rj = q[j] @ Qc.T
                F[wi, o + 6:o + 9] = Rj[0]
                F[wi, o + 9:o + 12] = Rj[1]
                F[wi, o + 12:o + 15] = w[j] * tau
                F[wi, o + 15] = 1.0
            g = 80
            F[wi, g:g + 3] = Qc @ v[p] * tau / L
            F[wi, g + 3:g + 6] = Qc @ (x[p] - mid[c]) / L
            F[wi, g + 6] = np.log10(inp.youngs[r] / 1e6)
            F[wi, g + 7] = inp.radius[r] / L
            Tb = L * L * np.sqrt(inp.density[r] * A / (inp.youngs[r] * I))
            F[wi, g + 8] = np.log10(tau / Tb)
            F[wi, g + 9] = inp.shear_coeff[r]
            F[wi, g + 10] = float(inp.bc_start[r])
            F[wi, g + 11] = c / n
            F[wi, g + 12] = 1.0 if wi == n else 0.0
            F[wi, g + 13] = amp / AMP_SCALE
            F[wi, g + 14] = np.sin(phase)
            F[wi, g + 15] = np.cos(phase)
        out.append(F)
    return np.concatenate(out)


def window_targets(inp, s0, s1, k):
    """Raw FP64 targets [sum(n+1), 12] and the loss mask (element outputs of
    end windows are masked)."""
    p0, v0, Q0, w0 = s0
    p1, v1, Q1, w1 = s1
    tau = k * inp.dt
    lh_all = (inp.rest_length if inp.rest_length is not None
              else np.concatenate([np.linalg.norm(np.diff(inp.position[ns], axis=0), axis=1)
                                   for ns, _ in rod_views(inp)]))
    T, Mk = [], []
    for r, (ns, es) in enumerate(rod_views(inp)):
        n = int(inp.n_elems[r])
        lh = lh_all[es]
        tgt = np.zeros((n + 1, N_OUT))
        msk = np.ones((n + 1, N_OUT))
        for wi in range(n + 1):
            c = min(wi, n - 1)
            p = wi if wi < n else n
            Qc = Q0[es][c]
            L = lh[c]
            tgt[wi, 0:3] = Qc @ (p1[ns][p] - p0[ns][p] - v0[ns][p] * tau) / L
            tgt[wi, 3:6] = Qc @ (v1[ns][p] - v0[ns][p]) * tau / L
            if wi < n:
                tgt[wi, 6:9] = _logvec(Qc @ Q1[es][c].T) - w0[es][c] * tau
                tgt[wi, 9:12] = (w1[es][c] - w0[es][c]) * tau
            else:
                msk[wi, 6:] = 0.0
        T.append(tgt)
        Mk.append(msk)
    return np.concatenate(T), np.concatenate(Mk)


def apply_deltas(inp, state, d, k):
    """State after one coarse step with raw predicted deltas d [sum(n+1), 12]:
    r_p += v_p tau + Q_c^T d[0:3] lh_c, v_p += Q_c^T d[3:6] lh_c / tau,
    Q_c <- P(exp(-[omega_c tau + d[6:9]]x) Q_c), omega_c += d[9:12] / tau (frames,
    velocities and angular velocities taken before the update), where P is the
    nearest rotation (orthogonal polar factor, from the SVD); clamped ends are
    left unchanged."""
    pos, vel, Q, om = (a.copy() for a in state)
    tau = k * inp.dt
    lh_all = (inp.rest_length if inp.rest_length is not None
              else np.concatenate([np.linalg.norm(np.diff(inp.position[ns], axis=0), axis=1)
                                   for ns, _ in rod_views(inp)]))
    row = 0
    for r, (ns, es) in enumerate(rod_views(inp)):
        n = int(inp.n_elems[r])
        Qr = state[2][es]
        v0, w0 = state[1][ns], state[3][es]
        x, v, q, w = pos[ns], vel[ns], Q[es], om[es]
        lh = lh_all[es]
        for wi in range(n + 1):
            c = min(wi, n - 1)
            p = wi if wi < n else n
            dd = d[row + wi]
            Qc = Qr[c]
            fixed_node = (p == 0 and inp.bc_start[r]) or (p == n and inp.bc_end[r])
            if not fixed_node:
                x[p] += v0[p] * tau + Qc.T @ dd[0:3] * lh[c]
                v[p] += Qc.T @ dd[3:6] * lh[c] / tau
            if wi < n:
                fixed_elem = (c == 0 and inp.bc_start[r]) or (c == n - 1 and inp.bc_end[r])
                if not fixed_elem:
                    q[c] = _nearest_rotation(_expmap(-(w0[c] * tau + dd[6:9])) @ Qr[c])
                    w[c] += dd[9:12] / tau
        pos[ns], vel[ns], Q[es], om[es] = x, v, q, w
        row += n + 1
    return pos, vel, Q, om


# ------------------------------------------------------------------ perturbation
# Counter-based N(0, 1) deviates: the splitmix64 output function (Steele, Lea and
# Flood, "Fast splittable pseudorandom number generators", 2014) hashes
# (seed, key); the top 24 and the low 24 bits give two uniforms in (0, 1), and
# the Box-Muller transform one normal deviate.

def _mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def gauss(seed, key):
    """N(0, 1) deviate for (seed, key) (arrays of keys allowed)."""
    h = _mix64(np.uint64(seed) ^ _mix64(key))
    u1 = ((h >> np.uint64(40)).astype(np.float64) + 0.5) / 16777216.0
    u2 = ((h & np.uint64(0xFFFFFF)).astype(np.float64) + 0.5) / 16777216.0
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def noise_key(r, j, kind, a):
    """Key of component a of quantity `kind` (0 position, 1 velocity,
    2 rotation, 3 angular velocity) at node or element j of rod r."""
    return (np.uint64(r) << np.uint64(32)) | (np.uint64(j) << np.uint64(4)) | np.uint64(3 * kind + a)


def perturb(inp, state, noise, seed, k):
    """Perturbed copy of a state: node positions += noise[0] lh g, node
    velocities += noise[1] lh / tau g, frames Q <- exp(-[noise[2] g]x) Q,
    angular velocities += noise[3] / tau g, g ~ N(0, 1) from gauss(seed, key)
    per component; lh of the node's own element (element n-1 for node n);
    clamped nodes and elements unchanged."""
    pos, vel, Q, om = (np.array(a, dtype=np.float64, copy=True) for a in state)
    tau = k * inp.dt
    lh_all = (inp.rest_length if inp.rest_length is not None
              else np.concatenate([np.linalg.norm(np.diff(inp.position[ns], axis=0), axis=1)
                                   for ns, _ in rod_views(inp)]))
    def g3(r, idx, kind):
        # [len(idx), 3] deviates for nodes / elements idx of rod r
        return np.stack([gauss(seed, noise_key(r, idx, kind, a)) for a in range(3)], axis=1)

    for r, (ns, es) in enumerate(rod_views(inp)):
        n = int(inp.n_elems[r])
        lh = lh_all[es]
        x, v, q, w = pos[ns], vel[ns], Q[es], om[es]
        nodes = np.array([j for j in range(n + 1)
                          if not ((j == 0 and inp.bc_start[r]) or (j == n and inp.bc_end[r]))], dtype=np.uint64)
        L = lh[np.minimum(nodes.astype(np.int64), n - 1)][:, None]
        ni = nodes.astype(np.int64)
        if noise[0] != 0:
            x[ni] += noise[0] * L * g3(r, nodes, 0)
        if noise[1] != 0:
            v[ni] += noise[1] * L / tau * g3(r, nodes, 1)
        elems = np.array([c for c in range(n)
                          if not ((c == 0 and inp.bc_start[r]) or (c == n - 1 and inp.bc_end[r]))], dtype=np.uint64)
        ei = elems.astype(np.int64)
        q[ei] = np.einsum("iab,ibc->iac", _expmap(-noise[2] * g3(r, elems, 2)), q[ei])
        w[ei] += noise[3] / tau * g3(r, elems, 3)
        pos[ns], vel[ns], Q[es], om[es] = x, v, q, w
    return pos, vel, Q, om


def judge_errors(inp, ref_state, state):
    """Per rod: max_j |dr_j| / L (against the plain reference) and the director
    orthonormality error max |Q Q^T - I| of `state`."""
    pr, pg = ref_state[0], state[0]
    Qg = state[2]
    errs = np.zeros((inp.n_rods, 2))
    for r, (ns, es) in enumerate(rod_views(inp)):
        L = np.sum(np.linalg.norm(np.diff(pr[ns], axis=0), axis=1))
        errs[r, 0] = np.linalg.norm(pg[ns] - pr[ns], axis=1).max() / L
        QQ = np.einsum("iab,icb->iac", Qg[es], Qg[es])
        errs[r, 1] = np.abs(QQ - np.eye(3)).max()
    return errs
