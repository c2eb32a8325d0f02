"""Benchmark of the rod step on one MI355X.

Workload: the ragged batch of 4096 free-free rods (16..256 elements,
556,994 elements in all), dt = 1e-5 s, damping 0.1; one bench step is one
rod_step call of 1000 position-Verlet steps (ceil(1000 / S) launches of the
persistent kernel replayed from a HIP graph, with the tile width and the
substeps per launch S chosen by the library's autotuner).  The headline value is FP64 element-steps/s; the
FP32 figure rides along in the same JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-surrogate] [--no-magnetic]
                  [--no-active] [--no-walls] [--no-contact] [--no-capsule] [--no-connected]

The magnetic carpet rides along as the "magnetic" object: 65,536 base-clamped
rods x 50 elements (FP32) turned by a rotating homogeneous field through their
programmed magnetization, timed like the headline and next to the same carpet
driven by its distributed couple.  The "active" object times 16,384 free
filaments x 50 elements under gravity and travelling-wave muscle moments in
both precisions, and the "walls" object the same filaments confined in a box
of six planar walls (penalty contact with Coulomb friction); the "contact"
object times a pile of crossed fibres in rod-rod contact (pairs in Verlet
lists rebuilt by a hash grid, one step per launch), and the "capsule" object the same pile with
fibres of aspect ratio 31 whose elements touch as capsules; the "connected"
object times millipede-like
bots of rods joined by point-wise and lateral spring-dashpot connections (224
bots, and 4096 to fill the GPU).

The learned coarse step rides along as the "surrogate" object: the network is
trained on 16,384 carpet rods (64 elements, 1.7e7 windows from 16 states of
plain trajectories, perturbed samples), then 262,144 carpet rods advance by
SURR_COARSE coarse steps of k = 32 with the plain integrator judging 1% of
them every 8 coarse steps; the same rods advance by the same simulated time
with the plain FP32 step.  Both rates are simulated seconds per wall second
for all rods (judge and fallback included); the end-to-end position error is
against the plain run.  The MLP's roofline is its fused inference kernel
timed alone on the same number of rows, against the BF16 dense MFMA peak.

Roofline: the step is plain ALU arithmetic once the rods' state stays on
chip for the 1000 substeps of a launch (1147 FLOP per byte of HBM traffic
in FP64), so `achieved` = algorithmic FLOP per launch / the launch's average
duration, measured with events on the launch stream, against the FP64
(FP32) vector peak.  ALGO_FLOP counts one element-step of the method
(two half drifts with Rodrigues rotations, strains, log-map curvature,
forces, the six couple terms and the kick) under +,-,* = 1, FMA = 2,
divide/sqrt/sin/cos/atan2 = 1.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rod element-steps/s (plain) and surrogate simulated-s/s at ≤1e-3 error"
ALGO_FLOP = 459                                  # per element-step (breakdown in the design notes)
ALGO_FLOP_MAG = 459 - 6 + 27                     # the external couple's 6 replaced by m x (Q b): 27
ALGO_FLOP_ACTIVE = 459 - 6 + 3 + 9               # no external couple; gravity 3; muscle moment 9
ALGO_BYTES = {"f64": 400, "f32": 204}            # HBM bytes per element per launch
MAG_BYTES = 12                                   # FP32 magnetization x rest length, read once per launch
MUSCLE_BYTES = {"f64": 32, "f32": 20}            # muscle amplitude x axis (T) and phase offset (FP64)
CONN_FLOP = 30                                   # one spring-dashpot force per connection and step
WALL_TEST_FLOP = 7                               # one node against one wall: n.x (5), minus offset and radius (2)
CONTACT_FLOP = 35                                # one node-wall contact: normal force 8, friction 15, sum 12
PEAK = {"f64": 78.6, "f32": 157.3}               # TFLOP/s, MI355X vector peaks
STEPS_PER_LAUNCH = 1000
SURR_K = 32
SURR_COARSE = 16                                 # two judge windows
# training recipe of the surrogate measurement (rod_surrogate_train): trajectories from 16,384 rods,
# 16 sampled states 1500 steps apart (2 states diverged in long runs; see the design notes)
SURR_TRAIN = dict(warmup_steps=2000, n_samples=16, sample_stride=1500, epochs=32, batch_rows=4096, lr=1e-3,
                  lr_min=1e-5, val_fraction=0.1, seed=7, noise=(1e-4, 1.5e-4, 3e-4, 6e-4))
MLP_FLOP = 2 * (96 * 256 + 256 * 256 * 2 + 256 * 12)   # per window
BF16_PEAK = 2500.0                               # TFLOP/s, dense MFMA
KERNEL_SRC = os.path.join(ROOT, "paper_2605_13766_amd", "csrc", "rod_kernels.hip")
CONTACT_SRC = os.path.join(ROOT, "paper_2605_13766_amd", "csrc", "contact_kernels.hip")


def kernel_hash(paths=(KERNEL_SRC,)) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(tag: str, tile_waves: int, substeps: int, paths=(KERNEL_SRC,)):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source in the same launch shape (else None).
    tag: {f64,f32}_ragged4096, f32_magnetic65536, {f64,f32}_active16384,
    {f64,f32}_activebox16384, {f64,f32}_millipede{224,4096} or f64_fibrepile16384
    (there: the whole step, contact pass included, per one-step launch)."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"rod_step_{tag}*_traffic.json"))):
        with open(path) as f:
            d = json.load(f)
        if (d.get("kernel_sha256_16") == kernel_hash(paths)
                and (d.get("tile_waves"), d.get("substeps")) == (tile_waves, substeps)):
            return d.get("hbm_bytes_per_launch")
    return None


def time_gpu(inp, precision, steps, warmup, tile_waves=0, substeps=0, algo_flop=ALGO_FLOP, extra_bytes=0,
             traffic_tag=None, probe=None, n_steps=STEPS_PER_LAUNCH):
    """Times `steps` bench steps after `warmup`.  algo_flop: FLOP per
    element-step, or a function of (probe before, probe after) when probe(batch)
    measures state the work depends on (outside the timed region)."""
    import torch
    from paper_2605_13766_amd import rod

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tuned = tile_waves == 0 or substeps == 0
        b = rod.RodBatch(inp, precision=precision, stream=stream, autotune=tuned, tile_waves=tile_waves,
                         substeps=substeps)
        info = b.info()
        info["tuning"] = b.tuning()
        for _ in range(warmup):
            b.step(n_steps, stream=stream)
        torch.cuda.synchronize()
        before = probe(b, stream) if probe else None
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            starts[k].record(stream)
            b.step(n_steps, stream=stream)
            ends[k].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
        after = probe(b, stream) if probe else None
        flags = b.flags(stream=stream)
        cstats = b.contact_stats(stream=stream) if getattr(inp, "rod_contact", 0) else None
        b.close()
    if flags.any():
        raise RuntimeError(f"{int(flags.sum())} rods became non-finite")
    el_steps = inp.n_elements * n_steps
    value = el_steps * steps / wall
    if probe:
        algo_flop = algo_flop(before, after)
    achieved = algo_flop * el_steps / (launch_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(traffic_tag or f"{precision}_ragged4096", info["tile_waves"], info["substeps"])
    return {
        "value": value,
        "ms_per_step": wall / steps * 1e3,
        "launch_ms": launch_ms,
        "info": info,
        "algo_flop": algo_flop,
        "probe": (before, after) if probe else None,
        "contact_stats": cstats,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK[precision],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK[precision],
            "traffic": traffic,
            "algorithmic_bytes_per_launch": (ALGO_BYTES[precision] + extra_bytes) * inp.n_elements,
        },
    }


def time_magnetic(steps, warmup, tile_waves=0, substeps=0):
    """The cilia carpet (65,536 base-clamped rods x 50 elements, FP32, dt 1e-6 s,
    autotuned) driven by the rotating magnetic field, next to the same carpet
    driven by its distributed couple: the cost of the magnetic couple."""
    from paper_2605_13766_amd import workloads as W
    mag = time_gpu(W.magnetic_carpet(), "f32", steps, warmup, tile_waves, substeps, algo_flop=ALGO_FLOP_MAG,
                   extra_bytes=MAG_BYTES, traffic_tag="f32_magnetic65536")
    drv = time_gpu(W.cilia_carpet(), "f32", steps, warmup, tile_waves, substeps, traffic_tag="none")
    return {
        "workload": "magnetic_carpet: 65,536 rods x 50 elements on a 256 x 256 grid, FP32, dt 1e-6 s, "
                    "field 10 mT rotating at 10 Hz, programmed magnetization 1.5e-3 A m, "
                    f"{STEPS_PER_LAUNCH} steps per launch",
        "value": mag["value"], "unit": "element-steps/s", "ms_per_step": mag["ms_per_step"],
        "launch_ms": mag["launch_ms"], "roofline": mag["roofline"],
        "tile_waves": mag["info"]["tile_waves"], "substeps_per_launch": mag["info"]["substeps"],
        "driven_carpet": {"value": drv["value"], "launch_ms": drv["launch_ms"],
                          "tile_waves": drv["info"]["tile_waves"], "substeps_per_launch": drv["info"]["substeps"]},
        "magnetic_over_driven_time": mag["launch_ms"] / drv["launch_ms"],
    }


def time_active(steps, warmup, tile_waves=0, substeps=0, precisions=("f64", "f32")):
    """Active filaments (16,384 free rods x 50 elements under gravity, driven by
    travelling muscle waves, dt 5e-5 s), both precisions, autotuned."""
    from paper_2605_13766_amd import workloads as W
    inp = W.active_filaments()
    out = {"workload": "active_filaments: 16,384 free rods x 50 elements, 1 m, gravity, travelling muscle "
                       f"moments (1 s period, wavelength 1 m), dt 5e-5 s, {STEPS_PER_LAUNCH} steps per launch",
           "unit": "element-steps/s"}
    for p in precisions:
        r = time_gpu(inp, p, steps, warmup, tile_waves, substeps, algo_flop=ALGO_FLOP_ACTIVE,
                     extra_bytes=MUSCLE_BYTES[p], traffic_tag=f"{p}_active16384")
        out[p] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "launch_ms": r["launch_ms"],
                  "roofline": r["roofline"], "tile_waves": r["info"]["tile_waves"],
                  "substeps_per_launch": r["info"]["substeps"]}
    return out


def wall_costs(inp, precision):
    """Algorithmic FLOP per element-step (a function of the node-wall contacts
    per element, measured before and after the timed steps) and extra bytes per
    element per launch of the boxed active filaments: the active step, every
    node tested against every wall, the contact force of every node-wall pair
    in contact (the mean of the two counts); bytes for the rod radii."""
    ne, R = inp.n_elements, inp.n_rods
    n_walls = len(inp.walls)
    base = ALGO_FLOP_ACTIVE + WALL_TEST_FLOP * n_walls * (ne + R) / ne

    def flop(before, after):
        return base + CONTACT_FLOP * 0.5 * (before + after)

    extra = MUSCLE_BYTES[precision] + 8 * R / ne
    return flop, extra


def contacts_per_element(inp):
    """probe for time_gpu: node-wall pairs in contact per element."""
    walls = np.asarray(inp.walls, dtype=np.float64)
    rad = np.repeat(np.asarray(inp.radius, dtype=np.float64), np.asarray(inp.n_elems) + 1)

    def probe(b, stream):
        pos = b.get_state(stream=stream)[0]
        delta = rad[:, None] - (pos @ walls[:, :3].T - walls[None, :, 3])
        return float(np.count_nonzero(delta > 0)) / inp.n_elements

    return probe


def time_walls(steps, warmup, tile_waves=0, substeps=0, precisions=("f64", "f32")):
    """Active filaments confined in a box: the active workload with six
    planar walls (penalty contact, Coulomb friction), both precisions."""
    from paper_2605_13766_amd import workloads as W
    inp = W.active_filaments(box=True)
    out = {"workload": f"active_box: 16,384 free rods x 50 elements in a 2 m box of {len(inp.walls)} walls "
                       f"(k {inp.wall_k:g} N/m^2, c {inp.wall_c:g} N s/m^2, mu {inp.wall_mu:g}), gravity, travelling "
                       f"muscle moments, dt 5e-5 s, {STEPS_PER_LAUNCH} steps per launch",
           "unit": "element-steps/s"}
    for p in precisions:
        flop, extra = wall_costs(inp, p)
        r = time_gpu(inp, p, steps, warmup, tile_waves, substeps, algo_flop=flop, extra_bytes=extra,
                     traffic_tag=f"{p}_activebox16384", probe=contacts_per_element(inp))
        out[p] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "launch_ms": r["launch_ms"],
                  "roofline": r["roofline"], "tile_waves": r["info"]["tile_waves"],
                  "substeps_per_launch": r["info"]["substeps"], "algorithmic_flop_per_element_step": r["algo_flop"],
                  "contacts_per_element": {"before": r["probe"][0], "after": r["probe"][1]}}
    return out


CONTACT_NODE_BYTES = 72                          # a contact pass: node position and velocity in, force out


def time_contact(steps, warmup, tile_waves=0, n_steps=STEPS_PER_LAUNCH, precisions=("f64", "f32")):
    """The fibre pile (16,384 fibres x 50 elements in 21 crossed layers on a
    floor, rod-rod contact over Verlet lists that the hash grid rebuilds when
    a node has moved more than half the skin), FP64 (the
    object's own figures) and FP32 (its "f32" member).  One step per launch, so
    the pass is HBM-bound: the roofline is bytes against the HBM peak,
    algorithmic bytes per step = the step's 400 (FP64) / 204 (FP32) per element
    (state in and out, constants) + 72 per node for the contact pass."""
    from paper_2605_13766_amd import workloads as W
    inp = W.fibre_pile()
    out = None
    for p in precisions:
        row = _time_contact_one(inp, p, steps, warmup, tile_waves, n_steps)
        if out is None:
            out = row
        else:
            out[p] = {k: row[k] for k in ("value", "ms_per_step", "ms_per_simulation_step", "tile_waves",
                                          "verlet_lists", "roofline")}
    return out


def time_capsule(steps, warmup, tile_waves=0, n_steps=STEPS_PER_LAUNCH, precisions=("f64", "f32")):
    """The capsule pile: 16,384 fibres of the paper's aspect ratio (31
    diameters, 20 elements of 3.1 radii) in 21 crossed layers on a floor,
    every element a capsule (segment contact, self-contact included), pairs
    kept in Verlet lists that the hash grid over element midpoints rebuilds
    when a node has moved more than half the skin.  Bytes as for the fibre
    pile: the step's per element plus 72 per node for the pass."""
    from paper_2605_13766_amd import workloads as W
    inp = W.capsule_pile()
    out = None
    for p in precisions:
        row = _time_contact_one(inp, p, steps, warmup, tile_waves, n_steps, tag="capsulepile16384")
        row["workload"] = (f"capsule_pile: {inp.n_rods:,} fibres x 20 elements (0.62 m, radius 1 cm, aspect ratio 31) "
                           f"in 21 crossed layers on a floor, capsule contact between elements (k {inp.wall_k:g} N/m, "
                           f"mu {inp.wall_mu:g}) over Verlet lists (skin 2 mm), gravity, dt 1e-5 s, one step per launch, "
                           f"{p.upper()}")
        if out is None:
            out = row
        else:
            out[p] = {k: row[k] for k in ("value", "ms_per_step", "ms_per_simulation_step", "tile_waves",
                                          "verlet_lists", "roofline")}
    return out


def _time_contact_one(inp, precision, steps, warmup, tile_waves, n_steps, tag="fibrepile16384"):
    # 4-wave tiles unless given: the tile widths differ by noise here (the contact pass does not depend on
    # them), and the counter runs behind the traffic figure were taken in that shape
    r = time_gpu(inp, precision, steps, warmup, tile_waves or 4, 1, traffic_tag="none", n_steps=n_steps)
    n_nodes = inp.n_elements + inp.n_rods
    step_s = r["launch_ms"] * 1e-3 / n_steps
    algo = ALGO_BYTES[precision] * inp.n_elements + CONTACT_NODE_BYTES * n_nodes
    achieved = algo / step_s / 1e9
    return {
        "workload": f"fibre_pile: {inp.n_rods:,} fibres x 50 elements (0.5 m, radius 1 cm) in 21 crossed layers on a "
                    f"floor, rod-rod contact (k {inp.wall_k:g} N/m, mu {inp.wall_mu:g}) over Verlet lists (skin 2 mm), "
                    f"gravity, dt 1e-5 s, one step per launch, {precision.upper()}",
        "unit": "element-steps/s",
        "value": r["value"], "ms_per_step": r["ms_per_step"], "steps_per_bench_step": n_steps,
        "ms_per_simulation_step": step_s * 1e3,
        "tile_waves": r["info"]["tile_waves"], "substeps_per_launch": r["info"]["substeps"],
        **({"verlet_lists": r["contact_stats"]} if r["contact_stats"] else {}),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                     "frac": achieved / 8000.0,
                     "traffic": traffic_from_profile(f"{precision}_{tag}", r["info"]["tile_waves"], 1,
                                                     (KERNEL_SRC, CONTACT_SRC)),
                     "algorithmic_bytes_per_step": algo},
    }


def connected_costs(inp, precision):
    """Algorithmic FLOP per element-step and extra bytes per element per launch of
    the millipede swarm: the plain step without the distributed couple, the
    magnetic couple on magnetized elements, one force per connection and step;
    bytes for the magnetization, the per-slot connection indices and the
    connection table (offsets, partners, k, c, l0)."""
    es = 8 if precision == "f64" else 4
    ne = inp.n_elements
    C = len(inp.conn_k)
    mag_frac = float(np.mean(np.any(inp.magnetization != 0, axis=1)))
    nodes = len({(int(r), int(j)) for pair_r, pair_j in zip(inp.conn_rod, inp.conn_node)
                 for r, j in zip(pair_r, pair_j)})
    flop = (ALGO_FLOP - 6 + 27 * mag_frac) + CONN_FLOP * C / ne
    extra = 3 * es + 8 + (4 * nodes + 2 * C * (4 + 3 * es)) / ne
    return flop, extra


def time_connected(steps, warmup, tile_waves=0, substeps=0, precisions=("f64", "f32"), bots_list=(224, 4096)):
    """The millipede swarm (rods joined by point-wise and lateral connections,
    magnetized legs in a rotating field): the paper's 224 bots, and 4096 bots
    that fill the GPU."""
    from paper_2605_13766_amd import workloads as W
    out = {"unit": "element-steps/s"}
    for bots in bots_list:
        inp = W.millipede_swarm(n_bots=bots)
        row = {"workload": f"millipede_swarm: {bots} bots of 26 rods (2 backbones x 20 + 24 legs x 8 elements, "
                           f"{inp.n_elements} elements), {len(inp.conn_k)} connections, rotating field, dt 1e-6 s, "
                           f"{STEPS_PER_LAUNCH} steps per launch"}
        for p in precisions:
            flop, extra = connected_costs(inp, p)
            r = time_gpu(inp, p, steps, warmup, tile_waves, substeps, algo_flop=flop, extra_bytes=extra,
                         traffic_tag=f"{p}_millipede{bots}")
            row[p] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "launch_ms": r["launch_ms"],
                      "roofline": r["roofline"], "tile_waves": r["info"]["tile_waves"],
                      "substeps_per_launch": r["info"]["substeps"], "algorithmic_flop_per_element_step": flop}
        out[f"bots{bots}"] = row
    return out


def cpu_baseline(inp, target_s=10.0):
    """The FP64 oracle on the host cores, on a seeded subset of the rods."""
    from oracle import rodoracle as ro
    threads = ro.max_threads()
    rng = np.random.default_rng(7)
    probe = inp.subset(rng.choice(inp.n_rods, size=64, replace=False))
    o = ro.Oracle(probe)
    t = time.perf_counter()
    o.step(100)
    rate = probe.n_elements * 100 / (time.perf_counter() - t)
    n_rods = int(np.clip(target_s * rate / (STEPS_PER_LAUNCH * inp.n_elements / inp.n_rods), 16,
                         inp.n_rods))
    sample = inp.subset(np.sort(rng.choice(inp.n_rods, size=n_rods, replace=False)))
    o = ro.Oracle(sample)
    t = time.perf_counter()
    o.step(STEPS_PER_LAUNCH)
    dt = time.perf_counter() - t
    # the same oracle on one thread: 100 steps of a sample sized for about 1.5 s
    k = int(np.clip(n_rods * 1.5 / max(dt * 0.1 * threads, 1e-9), 4, n_rods))
    one = inp.subset(np.sort(rng.choice(inp.n_rods, size=k, replace=False)))
    o1 = ro.Oracle(one)
    t = time.perf_counter()
    o1.step(100, n_threads=1)
    dt1 = time.perf_counter() - t
    o1.step(0, n_threads=threads)   # restores the thread count for later oracle calls
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": sample.n_elements * STEPS_PER_LAUNCH / dt,
        "unit": "element-steps/s",
        "cores": threads,
        "cpu_model": model,
        "one_thread_value": one.n_elements * 100 / dt1,
        "kind": "oracle",
        "sample": f"{n_rods} of the {inp.n_rods} rods ({sample.n_elements} elements), "
                  f"{STEPS_PER_LAUNCH} steps, FP64, {threads} OpenMP threads, {dt:.1f} s; one thread: {k} rods, "
                  f"100 steps, {dt1:.1f} s",
    }


def time_surrogate(n_coarse=None):
    """Train, then the coarse step with judge against the plain step on the
    262,144-rod carpet (see the module docstring).  n_coarse coarse steps
    (default SURR_COARSE), advanced in segments that end after 16, 32, 64, ...
    coarse steps, where the end-to-end error against the plain run is taken
    (outside the timed segments)."""
    n_coarse = n_coarse or SURR_COARSE
    import torch
    from paper_2605_13766_amd import rod
    from paper_2605_13766_amd import workloads as W

    out = {}
    t0 = time.perf_counter()
    tr = W.surrogate_training(n_rods=16384, n=64)
    btr = rod.RodBatch(tr, precision="f32")
    s = rod.Surrogate(k_substeps=SURR_K, seed=1)
    tdesc = dict(SURR_TRAIN)
    ep, val = s.train(btr, **tdesc)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    windows = int(tdesc["n_samples"] * (tr.n_elements + tr.n_rods))
    # minibatch rows processed: whole 4096-row batches of the 90% training share, every epoch;
    # forward + backward = 3 x the forward's FLOP per row (dA and dW each match the forward)
    rows = (int(0.9 * windows) // tdesc["batch_rows"]) * tdesc["batch_rows"] * tdesc["epochs"]
    out["train"] = {"rods": tr.n_rods, "windows": windows, "epochs": tdesc["epochs"],
                    "val_loss": float(val), "first_epoch_loss": float(ep[0]), "last_epoch_loss": float(ep[-1]),
                    "seconds": t_train,
                    "mlp_tflops": 3 * MLP_FLOP * rows / t_train / 1e12,
                    "note": "seconds include generating the trajectories; mlp_tflops divides the minibatch "
                            "MLP work by that whole time"}
    btr.close()
    del tr
    print("surrogate trained", out["train"], file=sys.stderr, flush=True)

    inp = W.surrogate_at_scale(n_rods=262144, n=64)
    judge = dict(judge_every=8, judge_fraction=0.01, max_pos_error=1e-3, max_orth_error=1e-5,
                 max_energy_error=5e-2, seed=11)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        pb = rod.RodBatch(inp, precision="f32", stream=stream, autotune=True)
        pinfo = pb.info()
        sb = rod.RodBatch(inp, precision="f32", stream=stream, tile_waves=pinfo["tile_waves"],
                          substeps=pinfo["substeps"])
        sb.step(2000, stream=stream)
        pb.step(2000 + SURR_K, stream=stream)
        s.step(sb, 1, stream=stream, **judge)        # allocations; both batches now at 2000 + k steps
        torch.cuda.synchronize()
        sim = n_coarse * SURR_K * inp.dt
        ends, e = [], 16
        while e < n_coarse:
            ends.append(e)
            e *= 2
        ends.append(n_coarse)
        ts = tp = 0.0
        st, trajectory, done = None, [], 0
        for end in ends:
            t = time.perf_counter()
            st_k = s.step(sb, end - done, stream=stream, **judge)
            torch.cuda.synchronize()
            ts += time.perf_counter() - t
            t = time.perf_counter()
            pb.step((end - done) * SURR_K, stream=stream)
            torch.cuda.synchronize()
            tp += time.perf_counter() - t
            done = end
            if st is None:
                st = dict(st_k)
            else:
                for key in ("coarse_steps", "judge_windows", "rods_judged", "rods_failed"):
                    st[key] += st_k[key]
                st["rods_plain"] = st_k["rods_plain"]
                for key in ("max_pos_error", "max_orth_error", "max_energy_error"):
                    st[key] = max(st[key], st_k[key])
            ps = pb.get_state(stream=stream)[0].reshape(-1, 65, 3)
            ss = sb.get_state(stream=stream, check=False)[0].reshape(-1, 65, 3)
            bad = (sb.flags(stream=stream) & rod.ROD_FLAG_NONFINITE) != 0
            err = np.linalg.norm(ss - ps, axis=2).max(axis=1) / 0.01
            ok = err[~bad]
            trajectory.append({"coarse_steps": end, "rods_nonfinite": int(bad.sum()),
                               "max": float(ok.max()), "median": float(np.median(ok)),
                               "frac_within_1e-3": float(np.mean(err <= 1e-3)), "rods_plain": st_k["rods_plain"],
                               "rods_failed": st["rods_failed"], "rods_judged": st["rods_judged"]})
        rng = np.random.default_rng(3)
        sample = rng.choice(inp.n_rods, size=64, replace=False)
        # the fused MLP kernel alone, on as many rows as the batch has windows
        rows = int(inp.n_elements + inp.n_rods)
        x = torch.randn((rows, 96), device="cuda").to(torch.bfloat16)
        y = torch.empty((rows, 12), device="cuda")
        s.forward(x, y, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            s.forward(x, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        mlp_ms = e0.elapsed_time(e1) / 3
        # one training step (forward keeping activations, backward, Adam) on the largest
        # workspace chunk, timed alone: the backward path's own throughput
        trows = 65536
        xt = x[:trows].contiguous()
        tt = torch.randn((trows, 12), device="cuda")
        s.train_step(xt, tt, lr=0.0, stream=stream, return_loss=False)
        e0.record(stream)
        for _ in range(5):
            s.train_step(xt, tt, lr=0.0, stream=stream, return_loss=False)
        e1.record(stream)
        torch.cuda.synchronize()
        train_ms = e0.elapsed_time(e1) / 5
        flags = sb.flags(stream=stream)
        sb.close()
        pb.close()
    s.close()
    if flags.any() and n_coarse == SURR_COARSE:
        raise RuntimeError(f"{int(flags.sum())} rods became non-finite under the coarse step")
    achieved = MLP_FLOP * rows / (mlp_ms * 1e-3) / 1e12
    out.update({
        "value": sim / ts,
        "unit": "simulated-s/s",
        "plain_value": sim / tp,
        "speedup": tp / ts,
        "workload": f"cilia carpet: {inp.n_rods} base-clamped rods x 64 elements, dt 1e-6 s, k = {SURR_K}, "
                    f"{n_coarse} coarse steps ({n_coarse * SURR_K} plain steps), judge every 8 on 1%, "
                    "thresholds 1e-3 position / 1e-5 orthonormality / 5e-2 strain energy",
        "ms_per_coarse_step": ts / n_coarse * 1e3,
        "plain_tile_waves": pinfo["tile_waves"],
        "plain_substeps_per_launch": pinfo["substeps"],
        "plain_ms_per_k_steps": tp / n_coarse * 1e3,
        "error": {"max": float(ok.max()), "median": float(np.median(ok)), "rods_nonfinite": int(bad.sum()),
                  "frac_within_1e-3": float(np.mean(err <= 1e-3)),
                  "sample64_max": float(err[sample].max())},
        "judge": st,
        "error_trajectory": trajectory,
        "mlp_roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK, "unit": "TFLOP/s",
                         "frac": achieved / BF16_PEAK, "rows": rows, "launch_ms": mlp_ms},
        "train_step_roofline": {"bound": "mfma", "achieved": 3 * MLP_FLOP * trows / (train_ms * 1e-3) / 1e12,
                                "peak": BF16_PEAK, "unit": "TFLOP/s",
                                "frac": 3 * MLP_FLOP * trows / (train_ms * 1e-3) / 1e12 / BF16_PEAK,
                                "rows": trows, "ms": train_ms,
                                "work": "forward with saved activations, backward (dA, split-reduction dW, bias "
                                        "sums), MSE gradient, Adam, BF16 refresh and fragment repack; "
                                        "3 x the forward's FLOP per row"},
    })
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="f64,f32")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-coarse", type=int, default=SURR_COARSE,
                    help="coarse steps of the surrogate measurement (errors taken after 16, 32, 64, ...)")
    ap.add_argument("--no-magnetic", action="store_true")
    ap.add_argument("--no-active", action="store_true")
    ap.add_argument("--no-connected", action="store_true")
    ap.add_argument("--no-walls", action="store_true")
    ap.add_argument("--no-contact", action="store_true")
    ap.add_argument("--no-capsule", action="store_true")
    ap.add_argument("--contact-steps", type=int, default=STEPS_PER_LAUNCH,
                    help="simulation steps per bench step of the contact workload (short runs for counters)")
    ap.add_argument("--connected-bots", default="224,4096", help="swarm sizes of the connected workload")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the headline batch (profiling runs of the other workloads; value is then null)")
    ap.add_argument("--tile-waves", type=int, default=0, help="fix the tile width (0: autotune)")
    ap.add_argument("--substeps", type=int, default=0, help="fix the substeps per launch (0: autotune)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (for scaling HBM counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        return 2

    import torch
    from paper_2605_13766_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20)
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 3}), flush=True)
        return 0
    print("generating the ragged 4096-rod batch", file=sys.stderr, flush=True)
    inp = W.ragged_batch(n_rods=4096)
    precs = args.precisions.split(",")
    res = {}
    for p in precs if not args.no_ragged else ():
        print(f"timing {p}", file=sys.stderr, flush=True)
        res[p] = time_gpu(inp, p, args.steps, args.warmup, args.tile_waves, args.substeps)
    if args.no_ragged:
        head = {"value": None, "ms_per_step": None, "info": {"tile_waves": None, "substeps": None, "n_tiles": None,
                                                              "tuning": []},
                "roofline": None, "launch_ms": None}
        precs = precs[:1]
    else:
        head = res[precs[0]]
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "element-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precs[0],
        "data": "synthetic",
        "config": {
            "workload": "ragged_batch: 4096 free-free rods, 16-256 elements, dt 1e-5 s, "
                        f"{STEPS_PER_LAUNCH} steps per launch",
            "n_rods": inp.n_rods,
            "n_elements": inp.n_elements,
            "steps_per_launch": STEPS_PER_LAUNCH,
            "tile_waves": head["info"]["tile_waves"],
            "substeps_per_launch": head["info"]["substeps"],
            "n_tiles": head["info"]["n_tiles"],
            "autotuner_trials": head["info"]["tuning"],
        },
        "roofline": head["roofline"],
        "launch_ms": head["launch_ms"],
    }
    for p in precs[1:]:
        line[p] = {"value": res[p]["value"], "unit": "element-steps/s",
                   "ms_per_step": res[p]["ms_per_step"], "launch_ms": res[p]["launch_ms"],
                   "roofline": res[p]["roofline"], "tile_waves": res[p]["info"]["tile_waves"],
                   "substeps_per_launch": res[p]["info"]["substeps"]}
    if not args.no_magnetic:
        print("timing the magnetic carpet", file=sys.stderr, flush=True)
        line["magnetic"] = time_magnetic(args.steps, args.warmup, args.tile_waves, args.substeps)
    if not args.no_active:
        print("timing the active filaments", file=sys.stderr, flush=True)
        line["active"] = time_active(args.steps, args.warmup, args.tile_waves, args.substeps,
                                     precisions=args.precisions.split(","))
    if not args.no_walls:
        print("timing the active filaments in a box", file=sys.stderr, flush=True)
        line["walls"] = time_walls(args.steps, args.warmup, args.tile_waves, args.substeps,
                                   precisions=args.precisions.split(","))
    if not args.no_contact:
        print("timing the fibre pile (rod-rod contact)", file=sys.stderr, flush=True)
        line["contact"] = time_contact(args.steps, args.warmup, args.tile_waves, args.contact_steps,
                                       precisions=args.precisions.split(","))
    if not args.no_capsule:
        print("timing the capsule pile (segment contact)", file=sys.stderr, flush=True)
        line["capsule"] = time_capsule(args.steps, args.warmup, args.tile_waves, args.contact_steps,
                                       precisions=args.precisions.split(","))
    if not args.no_connected:
        print("timing the millipede swarm", file=sys.stderr, flush=True)
        line["connected"] = time_connected(args.steps, args.warmup, args.tile_waves, args.substeps,
                                           precisions=args.precisions.split(","),
                                           bots_list=[int(x) for x in args.connected_bots.split(",")])
    if not args.no_cpu_baseline:
        print("timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(inp)
    if not args.no_surrogate:
        print("training and timing the learned coarse step", file=sys.stderr, flush=True)
        line["surrogate"] = time_surrogate(args.surrogate_coarse)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
