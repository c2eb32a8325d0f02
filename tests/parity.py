"""Error norms between a GPU state and the oracle's (tests only).

Per rod, then the maximum over rods:
  positions  max_j |dr_j| / L_rod
  velocities max_j |dv_j| / max(max_j |v_oracle|, L_rod / t_sim)
  directors  max |dQ| (entries)
  omega      max_i |dw_i| / max(max_i |w_oracle|, 1 / t_sim)
  energy     |dH| / (T + U), T + U floored at 1e-6 of the batch's largest
"""
from __future__ import annotations

import numpy as np


def rod_norms(inp, ref, got, t_sim):
    pr, vr, qr, wr = ref
    pg, vg, qg, wg = got
    out = {"pos": 0.0, "vel": 0.0, "dir": 0.0, "omega": 0.0}
    no, eo = inp.node_offset, inp.elem_offset
    for r, n in enumerate(inp.n_elems):
        nsl = slice(no[r], no[r] + n + 1)
        esl = slice(eo[r], eo[r] + n)
        L = np.sum(np.linalg.norm(np.diff(pr[nsl], axis=0), axis=1))
        out["pos"] = max(out["pos"], np.linalg.norm(pg[nsl] - pr[nsl], axis=1).max() / L)
        vs = max(np.abs(vr[nsl]).max(), L / t_sim)
        out["vel"] = max(out["vel"], np.abs(vg[nsl] - vr[nsl]).max() / vs)
        out["dir"] = max(out["dir"], np.abs(qg[esl] - qr[esl]).max())
        ws = max(np.abs(wr[esl]).max(), 1.0 / t_sim)
        out["omega"] = max(out["omega"], np.abs(wg[esl] - wr[esl]).max() / ws)
    return out


def energy_norm(e_ref, e_got):
    """|dH| / (T + U) per rod, max over rods, with T + U floored at 1e-6 of the
    batch's largest: a rod nearly at rest (1e-9 J against 0.2 J elsewhere in
    a batch) carries round-off of its stiff modes that is large against its own
    energy and negligible against the batch's."""
    H_r = e_ref.sum(axis=1)
    H_g = e_got.sum(axis=1)
    mech = e_ref[:, :4].sum(axis=1)
    scale = np.maximum(mech, max(1e-6 * float(mech.max()), 1e-300))
    return float(np.max(np.abs(H_g - H_r) / scale))


def oracle_pair(inp, steps):
    """The oracle's state after `steps`, and the same run started from positions
    moved by one ulp (same rest lengths): the round-off conditioning of the case."""
    from oracle import rodoracle as ro
    o = ro.Oracle(inp)
    p = ro.Oracle(inp)
    p.rest_length = o.rest_length.copy()
    p.pos = np.nextafter(p.pos, np.inf)
    p._mk()
    o.step(steps)
    p.step(steps)
    return o, p


def fp64_bars(inp, o, p, steps, floor=1e-10, factor=10.0):
    """Per-norm parity bar: max(floor, factor x the oracle's one-ulp sensitivity)."""
    sens = rod_norms(inp, o.state(), p.state(), steps * inp.dt)
    sens["energy"] = energy_norm(o.energy(), p.energy())
    return {k: max(floor, factor * v) for k, v in sens.items()}, sens
