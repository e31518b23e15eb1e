"""Throughput of the voxel-lattice time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload random_block_100]
                    [--precision 32|64] [--kernel fused|split] [--no-cpu]

Default workload: a 100^3 lattice whose cells are drawn from a seed as empty
(p = 0.1), soft 1 MPa (p = 0.45) or stiff 100 MPa (p = 0.45), density 1000,
resting 5 mm above a rigid floor with friction, gravity on.  A step is one
pass of the whole hot path (actuation, every bond, gather, floor/friction,
integrate) over the lattice.  The state is resident in HBM before timing
starts.  Prints one JSON line.

The metric is voxel-steps/s = filled voxels x steps / wall time of the K
timed steps (HIP events on the stream the kernels are launched on, with a
device synchronisation on both sides).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
# Algorithmic bytes per filled voxel-step: 13 state words read and written,
# material id read, flags read and written.
ALG_BYTES = {32: 13 * 4 * 2 + 3, 64: 13 * 8 * 2 + 3}


def build_workload(name):
    import workloads
    if name.startswith("random_block_"):
        n = int(name.split("_")[-1])
        return workloads.random_block(n=n, seed=2)
    if name.startswith("blob_lattice_"):
        n = int(name.split("_")[-1])
        w = workloads.blob_lattice(n=n, seed=3)
        return w
    if name.startswith("cube_"):
        n = int(name.split("_")[-1])
        return workloads.solid_cube(n, zeta_bond=0.5, gravity=9.81, floor_on=1)
    if name == "cantilever":
        return workloads.cantilever()
    raise SystemExit("unknown workload %s" % name)


def time_gpu(w, precision, kernel, steps, warmup, autotune=True):
    import torch
    import paper_1212_2845_amd as vx
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    s = vx.from_workload(w, precision=precision, kernel=kernel, stream=stream.cuda_stream)
    s.bind()
    if autotune and kernel == vx.KERNEL_FUSED:
        s.autotune(iters=3)
    nvox = s.counters()["voxels"]
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)                     # launches on `stream`, ends with a status poll
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return nvox, ms, s


def cpu_baseline(w, budget_s=12.0):
    """Oracle (FP64, one thread) on a bounded sample of the same workload."""
    import oracle
    o = oracle.Sim(w["grid"], w["materials"], **w["params"])
    if w.get("fixed") is not None:
        o.set_fixed(w["fixed"])
    if w.get("forces") is not None:
        o.set_forces(w["forces"])
    if w.get("velocity") is not None:
        o.set_velocity(w["velocity"])
    nvox = o.num_voxels
    o.step(1)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 2000:
            break
    return {"value": nvox * n / el, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d steps of the same %d-voxel lattice after 1 untimed step, FP64, one thread"
                      % (n, nvox)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="random_block_100")
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--kernel", default="fused", choices=["fused", "split"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling profiler byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import paper_1212_2845_amd as vx
    kernel = vx.KERNEL_FUSED if args.kernel == "fused" else vx.KERNEL_SPLIT
    w = build_workload(args.workload)
    print("[bench] workload %s precision %d kernel %s steps %d warmup %d"
          % (args.workload, args.precision, args.kernel, args.steps, args.warmup), file=sys.stderr, flush=True)
    nvox, ms, sim = time_gpu(w, args.precision, kernel, args.steps, args.warmup, not args.no_autotune)
    tile = sim.fused_tile() if kernel == vx.KERNEL_FUSED else None
    value = nvox * args.steps / (ms / 1e3)
    ms_step = ms / args.steps
    alg = ALG_BYTES[args.precision]
    achieved = alg * nvox / (ms_step / 1e3) / 1e9
    out = {
        "metric": "voxel-steps/s",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "cells": int(w["grid"].size), "voxels": int(nvox),
                   "kernel": args.kernel, "tile": tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_voxel_step": alg},
    }
    del sim
    if not args.no_fp64 and args.precision == 32:
        print("[bench] fp64 leg", file=sys.stderr, flush=True)
        n64, ms64, s64 = time_gpu(w, 64, kernel, args.steps, args.warmup, not args.no_autotune)
        tile64 = s64.fused_tile() if kernel == vx.KERNEL_FUSED else None
        del s64
        out["fp64"] = {"value": n64 * args.steps / (ms64 / 1e3), "ms_per_step": ms64 / args.steps, "tile": tile64,
                       "roofline_frac": ALG_BYTES[64] * n64 / (ms64 / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS}
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
