"""Error norms between a GPU state and the oracle's, and the parity bars (tests only).

Norms, per rod, then the maximum over rods:
  positions  max_j |dr_j| / L_rod
  velocities max_j |dv_j| / max(max_j |v_oracle|, L_rod / t_sim)
  directors  max |dQ| (entries)
  omega      max_i |dw_i| / max(max_i |w_oracle|, 1 / t_sim)
  energy     |dH| / (T + U), T + U floored at 1e-6 of the batch's largest

Bars:
  FP64  max(1e-10, 3 x the oracle's round-off conditioning), the conditioning
        being the largest divergence of the oracle from itself, after the same
        steps, over three starts whose positions differ from the real start by
        one ulp (every coordinate up; every coordinate down; every coordinate
        up or down by a seeded coin).  A rounding-order difference in any step
        perturbs the state by about that much, so no FP64 implementation
        other than the oracle itself can be asked for less.
  FP32  max(2^-20, 4 x the FP32 mirror's discrepancy), the mirror being the
        oracle's own step carried out in single precision (rod_oracle.c built
        with ORC_F32, state in the same edge form an FP32 implementation
        keeps); 2^-20 (16 FP32 rounding units) because discrepancies of a few
        units are decided by single roundings, where the ratio of two
        implementations' errors means nothing.
"""
from __future__ import annotations

import numpy as np

FP64_FLOOR = 1e-10
FP64_FACTOR = 3.0
FP32_FLOOR = 2.0 ** -20
FP32_FACTOR = 4.0
NORMS = ("pos", "vel", "dir", "omega", "energy")


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


def _one_ulp_starts(pos, seed=12345):
    """Three starting position arrays one ulp away from `pos` in every coordinate."""
    coin = np.random.default_rng(seed).integers(0, 2, size=pos.shape).astype(bool)
    yield np.nextafter(pos, np.inf)
    yield np.nextafter(pos, -np.inf)
    yield np.where(coin, np.nextafter(pos, np.inf), np.nextafter(pos, -np.inf))


def oracle_pair(inp, steps, draws=3):
    """The oracle's state after `steps`, and the same run from `draws` starts
    whose positions differ by one ulp (same rest lengths): the round-off
    conditioning of the case."""
    from oracle import rodoracle as ro
    o = ro.Oracle(inp)
    perts = []
    for k, start in enumerate(_one_ulp_starts(o.pos)):
        if k >= draws:
            break
        p = ro.Oracle(inp)
        p.rest_length = o.rest_length.copy()
        p.pos = np.ascontiguousarray(start)
        p._mk()
        perts.append(p)
    o.step(steps)
    for p in perts:
        p.step(steps)
    return o, perts


def fp64_bars(inp, o, perts, steps, floor=FP64_FLOOR, factor=FP64_FACTOR):
    """Per-norm FP64 bar: max(floor, factor x the largest one-ulp divergence)."""
    if not isinstance(perts, (list, tuple)):
        perts = [perts]
    sens = {k: 0.0 for k in NORMS}
    for p in perts:
        s = rod_norms(inp, o.state(), p.state(), steps * inp.dt)
        s["energy"] = energy_norm(o.energy(), p.energy())
        sens = {k: max(sens[k], s[k]) for k in NORMS}
    return {k: max(floor, factor * v) for k, v in sens.items()}, sens


def fp32_mirror(inp, steps):
    """The FP32 mirror of the oracle after `steps` from the same start."""
    from oracle import rodoracle as ro
    m = ro.Oracle32(inp)
    m.step(steps)
    return m


def fp32_bars(inp, o, m, steps, floor=FP32_FLOOR, factor=FP32_FACTOR):
    """Per-norm FP32 bar: max(floor, factor x the mirror's discrepancy from
    the FP64 oracle `o` after the same steps)."""
    disc = rod_norms(inp, o.state(), m.state(), steps * inp.dt)
    disc["energy"] = energy_norm(o.energy(), m.energy())
    return {k: max(floor, factor * v) for k, v in disc.items()}, disc


def bars_for(inp, precision, steps):
    """The FP64 oracle after `steps`, the bars for `precision`, and the
    quantity they derive from (one-ulp conditioning or mirror discrepancy)."""
    if precision == "f64":
        o, perts = oracle_pair(inp, steps)
        bars, base = fp64_bars(inp, o, perts, steps)
    else:
        from oracle import rodoracle as ro
        o = ro.Oracle(inp)
        o.step(steps)
        bars, base = fp32_bars(inp, o, fp32_mirror(inp, steps), steps)
    return o, bars, base


def check(norms, bars, keys=NORMS):
    """Names of the norms above their bars, with both values."""
    return {k: (norms[k], bars[k]) for k in keys if not norms[k] <= bars[k]}
