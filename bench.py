"""Benchmark of the rod step on one MI355X.

Workload: the ragged batch of 4096 free-free rods (16..256 elements,
556,994 elements in all), dt = 1e-5 s, damping 0.1; one bench step is one
rod_step call of 1000 position-Verlet steps (one persistent kernel launch
replayed from a HIP graph).  The headline value is FP64 element-steps/s; the
FP32 figure rides along in the same JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

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
ALGO_BYTES = {"f64": 400, "f32": 204}            # HBM bytes per element per launch
PEAK = {"f64": 78.6, "f32": 157.3}               # TFLOP/s, MI355X vector peaks
STEPS_PER_LAUNCH = 1000
KERNEL_SRC = os.path.join(ROOT, "paper_2605_13766_amd", "csrc", "rod_kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(precision: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"rod_step_{precision}_ragged4096_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def time_gpu(inp, precision, steps, warmup):
    import torch
    from paper_2605_13766_amd import rod

    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = rod.RodBatch(inp, precision=precision, stream=stream)
        info = b.info()
        for _ in range(warmup):
            b.step(STEPS_PER_LAUNCH, stream=stream)
        torch.cuda.synchronize()
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            starts[k].record(stream)
            b.step(STEPS_PER_LAUNCH, stream=stream)
            ends[k].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
        flags = b.flags(stream=stream)
        b.close()
    if flags.any():
        raise RuntimeError(f"{int(flags.sum())} rods became non-finite")
    el_steps = inp.n_elements * STEPS_PER_LAUNCH
    value = el_steps * steps / wall
    achieved = ALGO_FLOP * el_steps / (launch_ms * 1e-3) / 1e12
    traffic = traffic_from_profile(precision)
    return {
        "value": value,
        "ms_per_step": wall / steps * 1e3,
        "launch_ms": launch_ms,
        "info": info,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK[precision],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK[precision],
            "traffic": traffic,
            "algorithmic_bytes_per_launch": ALGO_BYTES[precision] * inp.n_elements,
        },
    }


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
    return {
        "value": sample.n_elements * STEPS_PER_LAUNCH / dt,
        "unit": "element-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n_rods} of the {inp.n_rods} rods ({sample.n_elements} elements), "
                  f"{STEPS_PER_LAUNCH} steps, FP64, {threads} OpenMP threads, {dt:.1f} s",
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="f64,f32")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        return 2

    import torch
    from paper_2605_13766_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    print("generating the ragged 4096-rod batch", file=sys.stderr, flush=True)
    inp = W.ragged_batch(n_rods=4096)
    precs = args.precisions.split(",")
    res = {}
    for p in precs:
        print(f"timing {p}", file=sys.stderr, flush=True)
        res[p] = time_gpu(inp, p, args.steps, args.warmup)
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
            "n_tiles": head["info"]["n_tiles"],
        },
        "roofline": head["roofline"],
        "launch_ms": head["launch_ms"],
    }
    for p in precs[1:]:
        line[p] = {"value": res[p]["value"], "unit": "element-steps/s",
                   "ms_per_step": res[p]["ms_per_step"], "launch_ms": res[p]["launch_ms"],
                   "roofline": res[p]["roofline"]}
    if not args.no_cpu_baseline:
        print("timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(inp)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
