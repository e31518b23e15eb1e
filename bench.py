"""Throughput of the voxel-lattice time step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload blob_lattice_256]
                    [--precision 32|64] [--kernel fused|split] [--no-cpu] [--no-cache-leg]
                    [--no-batch-leg] [--no-collision-leg] [--no-adjoint-leg]
                    [--no-paper-shape-leg] [--no-autotune] [--eager]

Headline workload: a 256^3 lattice (16.8M voxels, about 50M bonds) of 4
materials assigned from 64 seeded Voronoi blobs, E log-uniform in
[0.1, 100] MPa, CTE uniform in [0, 0.01]/K, a 5 Hz +/-20 K temperature
signal and self-collision on, in FP32.  A step is one pass of the whole hot
path (actuation, every bond, gather, contact, integrate, collision
bookkeeping) over the lattice.  Its state (872 MB per buffer) is far larger
than the GPU's 256 MB last-level cache, so the step streams from HBM.

Further legs: a 100^3 lattice of empty / soft / stiff cells dropped onto a
rigid floor with friction, in FP32 and FP64 (its state fits the last-level
cache, so it is reported as cache-resident); 4096 batched objects in one
persistent launch against the same objects one at a time; the iteration
rates of the paper's four self-collision schemes on a clapper; the
differentiable rollout of the 64 x 20^3 design lattice (forward + reverse
against the plain forward); one object's iteration rate on cubes of 8^3 to
40^3 on the GPU and the oracle (the paper's speed-versus-size sweep); the
oracle on one host core, and on a sample of the batched objects across the
host cores.

The state is resident on the GPU before timing starts.  Prints one JSON line.
voxel-steps/s = filled voxels x steps / time of the K timed steps: one
replay of a captured HIP graph of the K steps (vx_step_enqueue), timed with
HIP events on the replay stream, device synchronisation on both sides;
eager_value gives the same K steps as one vx_step call.  The roofline figure uses the step kernel's own average launch time,
measured the same way over dry-run launches that do not advance the state;
roofline.copy_probe is the rate of a plain 1 GiB device copy on the same GPU,
as context for the 8 TB/s peak.
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
        return workloads.random_block(n=int(name.split("_")[-1]), seed=2)
    if name.startswith("blob_lattice_"):
        return workloads.blob_lattice(n=int(name.split("_")[-1]), seed=3)
    if name.startswith("cube_"):
        return workloads.solid_cube(int(name.split("_")[-1]), zeta_bond=0.5, gravity=9.81, floor_on=1)
    if name == "cantilever":
        return workloads.cantilever()
    raise SystemExit("unknown workload %s" % name)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def time_gpu(w, precision, kernel, steps, warmup, autotune=True, tile=None, graph=True):
    """Returns a dict with voxels, ms for `steps` steps, the tile and the
    step kernel's own average launch time.  tile = (shape, zc) fixes the
    fused kernel's tile instead of autotuning it.  The timed steps are one
    captured HIP graph of `steps` vx_step_enqueue steps (an even count, so
    that the ping-pong state continues), replayed once after an untimed
    replay; eager_ms times the same number of steps as one vx_step call
    (and is the timed figure with graph=False, e.g. under a profiler's
    counter collection, which does not follow graph replays)."""
    import torch
    import paper_1212_2845_amd as vx
    torch.cuda.init()
    side = torch.cuda.Stream()
    s = vx.from_workload(w, precision=precision, kernel=kernel, stream=side.cuda_stream)
    s.bind()
    if tile is not None:
        s.set_fused_tile(*tile)
    elif autotune and kernel == vx.KERNEL_FUSED:
        s.autotune(iters=10)
    nvox = s.counters()["voxels"]
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(side)
    s.step(steps)                     # launches on `side`, ends with a status poll
    e1.record(side)
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1)
    ms = eager_ms
    if graph and steps % 2 == 0:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            s.step_enqueue(steps)
        g.replay()
        torch.cuda.synchronize()
        cs = torch.cuda.current_stream()     # replay() launches on the current stream
        e0.record(cs)
        g.replay()
        e1.record(cs)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        s.status()                        # raises if a replayed step went non-finite
        del g
    c = s.counters()
    kernel_ms = s.time_kernel(iters=max(10, min(steps, 50)))
    out = {"voxels": nvox, "ms": ms, "eager_ms": eager_ms, "kernel_ms": kernel_ms,
           "tile": s.fused_tile() if kernel == vx.KERNEL_FUSED else None,
           "collision": {"rebuilds": c["rebuilds"], "pairs": c["pairs"]}
           if w["params"].get("self_collision_on") else None}
    del s
    torch.cuda.empty_cache()
    return out


# Sources the fused step kernel is compiled from; profiler counters count
# for the current kernel only if they were taken on these exact files.
FUSED_SOURCES = ["vx_fused.hip", "vx_device.hpp", "vx_types.hpp", "vx_launch.hpp"]


def fused_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(ROOT, "paper_1212_2845_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, precision, tile, key=None):
    """HBM bytes per launch of the fused kernel (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy's readings) from profiles/traffic.json,
    or None when none was taken for this workload and tile on the current
    kernel source.  key names another entry (the batch kernel's, per step)."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if (tile is None and key is None) or not os.path.exists(p):
        return None
    with open(p) as fh:
        db = json.load(fh)
    e = db.get(key or "%s|f%d|tile%d:%d" % (workload, precision, tile["shape"], tile["zc"]))
    if e is None or e.get("src") != fused_source_hash():
        return None
    return e


# VALU issue peak of the chip: one wave64 instruction per CU per clock (no
# packed FP32), 256 CUs at 2.4 GHz, in lane-instructions per second.
VALU_PEAK_LANE_INSTR = 256 * 2.4e9 * 64


def measured_valu(workload, precision, tile):
    """VALU lane-instructions per voxel-step of the fused kernel (rocprofv3
    SQ_INSTS_VALU x 64 / voxels) from profiles/valu.json, or None when none
    was taken for this workload and tile on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "valu.json")
    if tile is None or not os.path.exists(p):
        return None
    with open(p) as fh:
        db = json.load(fh)
    e = db.get("%s|f%d|tile%d:%d" % (workload, precision, tile["shape"], tile["zc"]))
    if e is None or e.get("src") != fused_source_hash():
        return None
    return e


def roofline(precision, nvox, kernel_ms, workload=None, tile=None, kernel="k_fused", traffic_key=None):
    alg = ALG_BYTES[precision]
    achieved = alg * nvox / (kernel_ms / 1e3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kernel,
           "kernel_ms": kernel_ms, "alg_bytes_per_voxel_step": alg, "voxels_per_launch": nvox}
    t = measured_traffic(workload, precision, tile, traffic_key) if workload else None
    if t is not None:
        out["traffic"] = t["traffic"]
        out["traffic_unit"] = "bytes per launch" if traffic_key is None else "bytes per step"
        out["traffic_over_algorithmic"] = t["traffic"] / (alg * nvox)
        out["traffic_profile"] = "profiles/" + t["profile"]
    v = measured_valu(workload, precision, tile) if workload else None
    if v is not None:
        rate = v["per_voxel_step"] * nvox / (kernel_ms / 1e3)
        out["alu"] = {"achieved": rate / 1e12, "peak": VALU_PEAK_LANE_INSTR / 1e12,
                      "unit": "T VALU lane-instructions/s", "frac": rate / VALU_PEAK_LANE_INSTR,
                      "valu_per_voxel_step": v["per_voxel_step"], "profile": "profiles/" + v["profile"],
                      "note": "the same launch against the chip's VALU issue rate; the step kernel is "
                              "VALU-bound before it is HBM-bound"}
    return out


def time_batch(count, steps, one_by_one_sample=256, one_by_one_steps=100):
    """Batched objects: one persistent launch for all objects vs the same
    objects stepped one at a time through the single-lattice path."""
    import torch
    import paper_1212_2845_amd as vx
    import workloads
    objs = workloads.batch_objects(count=count, seed=4, steps=steps)
    mats, params = objs[0]["materials"], objs[0]["params"]
    stream = torch.cuda.current_stream()
    b = vx.Batch([o["grid"] for o in objs], mats, precision=32, stream=stream.cuda_stream, **params)
    b.bind()
    n_wg = b.autotune(steps=20)
    tile_rule = b.tile(0)[0]
    nvox = b.counters()["voxels"]
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    del b
    torch.cuda.empty_cache()
    batched = nvox * steps / (ms / 1e3)
    result = {"workload": "batch_objects_%d" % count, "objects": count, "voxels": nvox, "steps": steps,
              "dtype": "f32", "value": batched, "ms": ms, "workgroups": n_wg, "tile_rule": tile_rule,
              "roofline": dict(roofline(32, nvox, ms / steps, "batch_objects_%d" % count, kernel="k_batch",
                                        traffic_key="batch_objects_%d|f32|k_batch" % count),
                               note="kernel_ms is per step: one persistent launch runs all steps")}
    if one_by_one_sample <= 0:
        return result
    # one at a time: every k-th object of the same batch (a sample with the
    # batch's mix of sizes and classes), each its own lattice, every object's
    # steps recorded into one HIP graph (stream capture of vx_step_enqueue)
    # and replayed, so that launch overhead is not counted
    stride = max(1, count // one_by_one_sample)
    sample = objs[::stride][:one_by_one_sample]
    side = torch.cuda.Stream()
    sims = [vx.from_workload(o, precision=32, stream=side.cuda_stream) for o in sample]
    for s in sims:
        s.bind()
        s.step(2)
    nvox1 = sum(s.counters()["voxels"] for s in sims)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for s in sims:
            s.step_enqueue(one_by_one_steps)
    graph.replay()
    torch.cuda.synchronize()
    # replay() launches on the current stream: time it there
    cs = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(cs)
    graph.replay()
    e1.record(cs)
    torch.cuda.synchronize()
    ms1 = e0.elapsed_time(e1)
    for s in sims:
        s.status()
    # the same loop without graphs, one vx_step call per object
    t0 = time.perf_counter()
    for s in sims:
        s.step(one_by_one_steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del graph, sims
    torch.cuda.empty_cache()
    single = nvox1 * one_by_one_steps / (ms1 / 1e3)
    single_eager = nvox1 * one_by_one_steps / el
    return dict(result, **{
            "one_by_one": {"value": single, "objects": len(sample), "steps": one_by_one_steps,
                           "eager_value": single_eager,
                           "voxels": nvox1,
                           "note": "a sample of the batch: every %d-th of its %d objects (%d objects, %d voxels, "
                                   "the batch's mix of sizes), %d steps each, each stepped alone through the "
                                   "fused single-lattice path; value: all these objects' steps in one captured HIP "
                                   "graph, replayed; eager_value: one vx_step call per object; the speedup compares "
                                   "voxel-step rates (batch: all objects, %d steps)"
                                   % (stride, count, len(sample), nvox1, one_by_one_steps, steps)},
            "speedup": batched / single})


def time_adjoint(steps=5000, K=100):
    """Differentiable rollout of the design lattice (64 blocks of 20^3,
    per-voxel moduli and phases, FP32) from rest: a plain forward of `steps`
    steps in parameter mode vs the forward with checkpoints plus the reverse
    run (segment recompute included) of the same rollout on a fresh handle,
    loss = mean x displacement."""
    import numpy as np
    import torch
    import paper_1212_2845_amd as vx
    import workloads
    stream = torch.cuda.current_stream()

    def make(w):
        s = vx.from_workload(w, precision=32, stream=stream.cuda_stream)
        s.set_stiffness(w["E"])
        s.bind()
        return s

    # warm-up of every kernel on a small lattice of the same kind
    ws = workloads.design_lattice(count=4, size=8, steps=40)
    s = make(ws)
    s.step(5)
    s.grad_bind(40, 10)
    s.grad_forward(40)
    s.grad_backward(dL_du=np.ones((ws["grid"].size, 3)), initial_state=False)
    del s
    w = workloads.design_lattice(steps=steps)
    filled = w["grid"].reshape(-1) > 0
    nvox = int(filled.sum())
    wu = np.zeros((w["grid"].size, 3))
    wu[filled, 0] = 1.0 / nvox
    s = make(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    del s
    # the same lattice with the palette's moduli (no per-voxel constants to
    # derive): the fastest plain forward of this lattice
    s = vx.from_workload(w, precision=32, stream=stream.cuda_stream)
    s.bind()
    s.step(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_fused = time.perf_counter() - t0
    del s
    s = make(w)
    gbytes = s.grad_bind(steps, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.grad_forward(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = s.grad_backward(dL_du=wu, initial_state=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del s
    torch.cuda.empty_cache()
    t_fa = t2 - t0
    # the same rollout with the full tape (K = 1: every step's state and bond
    # sums stored by the forward run, nothing recomputed), when it fits the
    # free HBM
    tape = None
    s = make(w)
    need = s.grad_workspace_bytes(steps, 1)
    free = torch.cuda.mem_get_info()[0]
    if need < 0.9 * free:
        s.grad_bind(steps, 1)
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        s.grad_forward(steps)
        torch.cuda.synchronize()
        u1 = time.perf_counter()
        gt = s.grad_backward(dL_du=wu, initial_state=False)
        torch.cuda.synchronize()
        u2 = time.perf_counter()
        same = all(np.array_equal(gt[k], g[k]) for k in ("E", "rho", "phase", "amp"))
        tape = {"grad_workspace_bytes": int(need), "grad_forward_s": u1 - u0, "grad_backward_s": u2 - u1,
                "fwd_adj_over_fwd": (u2 - u0) / t_fwd, "fwd_adj_over_fused_fwd": (u2 - u0) / t_fused,
                "gradients_equal_to_checkpointed": bool(same)}
    else:
        tape = {"skipped": "tape of %d bytes does not fit %d free bytes" % (need, free)}
    del s
    torch.cuda.empty_cache()
    return {"workload": w["name"], "voxels": nvox, "cells": int(w["grid"].size), "steps": steps,
            "checkpoint_every": K, "dtype": "f32", "grad_workspace_bytes": int(gbytes),
            "forward_s": t_fwd, "grad_forward_s": t1 - t0, "grad_backward_s": t2 - t1,
            "fwd_adj_over_fwd": t_fa / t_fwd,
            "fused_forward_s": t_fused, "fwd_adj_over_fused_fwd": t_fa / t_fused, "target_fwd_adj_over_fwd": 4.0,
            "value": nvox * steps / t_fa, "unit": "voxel-steps/s (forward + reverse)", "tape_K1": tape,
            "grad_E_absmax": float(np.abs(g["E"]).max()), "grad_phase_absmax": float(np.abs(g["phase"]).max()),
            "note": "forward_s: the plain forward in parameter mode (per-voxel moduli) through the fused step "
                    "kernel, which the recorded forward and the segment recompute also run; fused_forward_s: the "
                    "same lattice with the palette's moduli; the target is fwd+adj <= 4 x fwd; wall time with host "
                    "synchronisation at each checkpoint and the host copies of the adjoint in and the gradients "
                    "out; the reverse run returns the per-voxel modulus, density, phase and amplitude gradients (the "
                    "design loop's), not those of the initial state"}


def time_adjoint_contact(steps=1000, K=100, pairs=(8, 8, 8)):
    """Differentiable rollout through voxel-voxel contact: the colliding
    bodies (pairs of free bodies driven into each other, self-collision on,
    FP32) in parameter mode, a plain forward of `steps` steps against the
    forward with checkpoints every K steps plus the reverse run (candidate
    lists built where the forward rebuilt them, the contact forces' reverse
    applied), and the same with the full tape; loss = mean x
    displacement."""
    import numpy as np
    import torch
    import paper_1212_2845_amd as vx
    import workloads
    stream = torch.cuda.current_stream()
    w, _ = workloads.colliding_bodies(pairs=pairs, steps=steps)
    filled = w["grid"].reshape(-1) > 0
    nvox = int(filled.sum())
    E = np.array([w["materials"][m]["E"] if m else 0.0 for m in w["grid"].reshape(-1)])
    wu = np.zeros((w["grid"].size, 3))
    wu[filled, 0] = 1.0 / nvox

    def make():
        s = vx.from_workload(w, precision=32, stream=stream.cuda_stream)
        s.set_stiffness(E)
        s.bind()
        s.write_state(**w["state"])
        return s

    # warm-up of every kernel on a short rollout
    s = make()
    s.grad_bind(20, 10)
    s.grad_forward(20)
    s.grad_backward(dL_du=wu, initial_state=False)
    del s
    s = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    rebuilds = s.counters()["rebuilds"]
    del s
    out = {"workload": w["name"], "voxels": nvox, "cells": int(w["grid"].size), "steps": steps, "dtype": "f32",
           "forward_s": t_fwd, "rebuilds": rebuilds}
    grads = {}
    for k in (K, 1):
        s = make()
        s.grad_bind(steps, k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.grad_forward(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        grads[k] = s.grad_backward(dL_du=wu, initial_state=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out["K%d" % k] = {"grad_forward_s": t1 - t0, "grad_backward_s": t2 - t1,
                          "fwd_adj_over_fwd": (t2 - t0) / t_fwd}
        del s
        torch.cuda.empty_cache()
    out["gradients_equal_K%d_K1" % K] = bool(all(np.array_equal(grads[K][q], grads[1][q])
                                                 for q in ("E", "rho", "phase", "amp")))
    out["note"] = ("wall time with host synchronisation; the reverse run (and the segment recompute with K > 1) "
                   "builds candidate lists where the forward's horizon rule rebuilt them and at each segment's "
                   "first step")
    return out


def time_collision_schemes(steps=5000, graph=True, w=None):
    """Iteration rates of the self-collision schemes of the paper's Table 3
    (candidates from all voxels or the surface; rebuilt every step or by the
    horizon rule) on the clapper (or on workload w), FP32: wall time of
    `steps` steps as one vx_step call (host launches included), and the same
    steps from the same start replayed from one captured HIP graph (device
    time; the rebuild decisions are taken on the device, so the graph runs
    the same work)."""
    import torch
    import paper_1212_2845_amd as vx
    import workloads
    if w is None:
        w = workloads.clapper(steps=steps)
    out = {"workload": w["name"], "voxels": int((w["grid"] > 0).sum()), "steps": steps, "dtype": "f32",
           "unit": "iterations/s",
           "note": "NAME: wall time of vx_step over the steps, host launches included; NAME graph: one replay "
                   "of the same steps captured as a HIP graph; NAME rebuilds: candidate-list rebuilds"}
    rates = {}
    side = torch.cuda.Stream()

    def make(all_voxels, every):
        sim = vx.from_workload(w, precision=32, stream=side.cuda_stream)
        sim.set_collision_mode(all_voxels, every)
        if w.get("state") is not None:
            sim.write_state(**w["state"])
        sim.step(10)
        return sim

    for all_voxels, every, name in [(1, 1, "all+every"), (0, 1, "surf+every"), (1, 0, "all+horizon"),
                                    (0, 0, "surf+horizon")]:
        s = make(all_voxels, every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        rates[name] = steps / (time.perf_counter() - t0)
        c = s.counters()
        rates[name + " rebuilds"] = c["rebuilds"]
        rates[name + " pairs"] = c["pairs"]
        del s
        if graph and steps % 2 == 0:
            s = make(all_voxels, every)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                s.step_enqueue(steps)
            cs = torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(cs)
            g.replay()
            e1.record(cs)
            torch.cuda.synchronize()
            s.status()
            rates[name + " graph"] = steps / (e0.elapsed_time(e1) / 1e3)
            del g, s
    out["rates"] = rates
    return out


def copy_probe(mib=1024, reps=5):
    """Achievable HBM rate on this device: a plain device-to-device copy of
    mib MiB (read once, written once), best of reps, timed with HIP events."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 1e30
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": 2 * n * 4 / (best / 1e3) / 1e9, "bytes_each_way": n * 4,
            "note": "torch device copy, best of %d; context for the 8 TB/s peak" % reps}


def time_paper_shape(ns=(8, 16, 24, 32, 40), steps=2000, cpu_budget_s=1.5):
    """The paper's speed-versus-size sweep: cubic blocks of one 1 MPa
    material, bottom layer fixed, gravity and bond damping on.  Iterations
    per second of one object on the GPU (one vx_step call, and the same steps
    replayed from one captured HIP graph) and on the oracle (FP64, one
    thread), beside the paper's figure for a 4000-voxel object."""
    import numpy as np
    import torch
    import oracle
    import paper_1212_2845_amd as vx
    import workloads
    rows = []
    for n in ns:
        w = workloads.solid_cube(n, E=1e6, gravity=9.81, zeta_bond=0.5)
        _, _, z = workloads.cell_coords(w["grid"].shape)
        w["fixed"] = (z == 0).astype(np.uint8)
        side = torch.cuda.Stream()
        sim = vx.from_workload(w, precision=32, stream=side.cuda_stream)
        sim.bind()
        sim.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        eager = steps / (time.perf_counter() - t0)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            sim.step_enqueue(steps)          # even: replays continue the state
        graph.replay()
        torch.cuda.synchronize()
        cs = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(cs)
        graph.replay()
        e1.record(cs)
        torch.cuda.synchronize()
        sim.status()
        graph_its = steps / (e0.elapsed_time(e1) / 1e3)
        del graph, sim
        o = oracle.Sim(w["grid"], w["materials"], **w["params"])
        o.set_fixed(w["fixed"])
        o.step(1)
        t0 = time.perf_counter()
        k = 0
        while True:
            o.step(1)
            k += 1
            el = time.perf_counter() - t0
            if el > cpu_budget_s or k >= 500:
                break
        rows.append({"n": n, "voxels": n ** 3, "gpu_its": eager, "gpu_graph_its": graph_its,
                     "oracle_its": k / el, "gpu_graph_voxel_steps": graph_its * n ** 3,
                     "oracle_voxel_steps": k / el * n ** 3})
    torch.cuda.empty_cache()
    return {"workload": "solid cubes n^3, 1 MPa, bottom layer fixed, gravity, zeta_bond 0.5", "dtype_gpu": "f32",
            "steps_gpu": steps, "rows": rows,
            "paper": {"its": 122, "voxels": 4000, "voxel_steps": 488000,
                      "hardware": "one thread of a 2.67 GHz Core i7", "note": "context only"}}


def host_cpu():
    """Model name of the host CPU, as /proc/cpuinfo gives it."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def crop_workload(w, n):
    """The lower n^3 corner of a workload's lattice, with its materials and
    parameters (per-cell inputs cropped alike): a sample of the same
    workload small enough for the oracle."""
    g = w["grid"]
    nz, ny, nx = g.shape
    cz, cy, cx = min(n, nz), min(n, ny), min(n, nx)
    out = dict(w)
    out["grid"] = np.ascontiguousarray(g[:cz, :cy, :cx])
    for k in ("fixed", "amp", "phase"):
        if w.get(k) is not None:
            out[k] = np.ascontiguousarray(np.asarray(w[k]).reshape(nz, ny, nx)[:cz, :cy, :cx].reshape(-1))
    for k in ("forces", "velocity"):
        if w.get(k) is not None:
            out[k] = np.ascontiguousarray(np.asarray(w[k]).reshape(nz, ny, nx, 3)[:cz, :cy, :cx].reshape(-1, 3))
    out["name"] = "%s cropped to %dx%dx%d" % (w["name"], cx, cy, cz)
    return out


def cpu_baseline(w, budget_s=12.0, note="", crop=None):
    """The oracle (FP64, one thread) on a bounded sample of the workload:
    the first steps of the whole lattice, or of its lower crop^3 corner when
    crop is given (the oracle's brute-force candidate search is quadratic in
    the surface voxels, so the full 256^3 lattice is out of its reach)."""
    import oracle
    if crop is not None:
        w = crop_workload(w, crop)
    o = oracle.Sim(w["grid"], w["materials"], **w["params"])
    if w.get("fixed") is not None:
        o.set_fixed(w["fixed"])
    if w.get("forces") is not None:
        o.set_forces(w["forces"])
    if w.get("velocity") is not None:
        o.set_velocity(w["velocity"])
    if w.get("amp") is not None or w.get("phase") is not None:
        o.set_actuation(w.get("amp"), w.get("phase"))
    nvox = o.num_voxels
    t0 = time.perf_counter()
    o.step(1)                        # builds the collision candidates when self-collision is on
    first_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 2000:
            break
    return {"value": nvox * n / el, "unit": "voxel-steps/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "sample": "%d steps of the %d-voxel %s lattice after 1 untimed step (%.1f s, including the "
                      "oracle's first candidate search when self-collision is on), FP64, one thread%s"
                      % (n, nvox, w["name"], first_s, note)}


def cpu_batch_baseline(count, sample_every=32, steps=60):
    """The oracle (FP64) on a sample of the batched objects, one object per
    thread across the host's cores (at most 16; the C oracle releases the GIL
    while it steps), and the single-core rate of the same work."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import workloads
    objs = workloads.batch_objects(count=count, seed=4, steps=steps)[::sample_every]
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu))

    def make(o):
        return oracle.Sim(o["grid"], o["materials"], **o["params"])

    def run(sim):
        t0 = time.perf_counter()
        sim.step(steps)
        return time.perf_counter() - t0

    with ThreadPoolExecutor(threads) as ex:
        sims = list(ex.map(make, objs))
        nvox = sum(sim.num_voxels for sim in sims)
        t0 = time.perf_counter()
        busy = sum(ex.map(run, sims))
        wall = time.perf_counter() - t0
    return {"value": nvox * steps / wall, "unit": "voxel-steps/s", "cores": threads, "kind": "oracle",
            "host": host_cpu(),
            "single_core_value": nvox * steps / busy,
            "sample": "one in every %d of the %d objects (%d objects, %d voxels), %d steps each, FP64, one object "
                      "per thread on %d threads; single_core_value: the same voxel-steps over the summed "
                      "per-object step times" % (sample_every, count, len(objs), nvox, steps, threads)}


def lattice_leg(w, precision, r, steps, kernel_name):
    """JSON block of one timed lattice run."""
    return {"workload": w["name"], "dtype": "f32" if precision == 32 else "f64",
            "value": r["voxels"] * steps / (r["ms"] / 1e3), "ms_per_step": r["ms"] / steps, "tile": r["tile"],
            "kernel": kernel_name, "eager_value": r["voxels"] * steps / (r["eager_ms"] / 1e3),
            "cache_resident": 2 * int(w["grid"].size) * 13 * (4 if precision == 32 else 8) < 256e6,
            "roofline": roofline(precision, r["voxels"], r["kernel_ms"], w["name"], r["tile"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="blob_lattice_256")
    ap.add_argument("--precision", type=int, default=32, choices=[32, 64])
    ap.add_argument("--kernel", default="fused", choices=["fused", "split"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-cache-leg", action="store_true",
                    help="skip the cache-resident 100^3 random block (FP32 and FP64)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batch-leg", action="store_true")
    ap.add_argument("--no-collision-leg", action="store_true")
    ap.add_argument("--no-adjoint-leg", action="store_true")
    ap.add_argument("--no-paper-shape-leg", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="no graph replays: the lattice legs' K steps as one vx_step call, and the collision "
                         "leg's eager rates only (for profiler counter runs, which do not follow graph replays)")
    ap.add_argument("--adjoint-steps", type=int, default=5000)
    ap.add_argument("--adjoint-contact-steps", type=int, default=1000,
                    help="steps of the rollout through contact in the adjoint leg (0: skip it)")
    ap.add_argument("--batch-objects", type=int, default=4096)
    ap.add_argument("--one-by-one-sample", type=int, default=256,
                    help="objects in the one-at-a-time comparison of the batched leg (0 skips it, e.g. "
                         "under profiler counter collection, which does not follow graph launches)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--cpu-crop", type=int, default=32,
                    help="edge of the lower corner of a self-colliding lattice the oracle baseline runs on")
    ap.add_argument("--tile", default=None, metavar="SHAPE:ZC",
                    help="fix the fused tile of the first leg (shape index, z chunk) instead of autotuning")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
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
    import paper_1212_2845_amd as vx
    kernel = vx.KERNEL_FUSED if args.kernel == "fused" else vx.KERNEL_SPLIT
    autotune = not args.no_autotune
    tile = tuple(int(v) for v in args.tile.split(":")) if args.tile else None

    w = build_workload(args.workload)
    log("workload %s precision %d kernel %s steps %d warmup %d"
        % (args.workload, args.precision, args.kernel, args.steps, args.warmup))
    use_graph = not args.eager and args.steps % 2 == 0
    r = time_gpu(w, args.precision, kernel, args.steps, args.warmup, autotune, tile, graph=use_graph)
    state_bytes = int(w["grid"].size) * 13 * (4 if args.precision == 32 else 8)
    # the headline is the plain vx_step call; the replay of the same steps
    # captured as a HIP graph is reported beside it (on this lattice its
    # seven dependent nodes per step run slower than the eager launches)
    out = {
        "metric": "voxel-steps/s",
        "value": r["voxels"] * args.steps / (r["eager_ms"] / 1e3),
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["eager_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "cells": int(w["grid"].size), "voxels": int(r["voxels"]),
                   "kernel": args.kernel, "tile": r["tile"], "state_bytes": state_bytes,
                   "self_collision": bool(w["params"].get("self_collision_on")),
                   "cache_resident": 2 * state_bytes < 256e6},
        "roofline": roofline(args.precision, r["voxels"], r["kernel_ms"], w["name"], r["tile"]),
        "timing": {"method": "one vx_step call of the K steps (host launches included), HIP events on its "
                             "stream, device synchronisation on both sides",
                   "graph_value": r["voxels"] * args.steps / (r["ms"] / 1e3) if use_graph else None,
                   "graph_method": "one replay of the K steps captured as a HIP graph, after an untimed replay"},
    }
    if r["collision"] is not None:
        out["collision"] = dict(r["collision"], note="candidate-list rebuilds since creation (warm-up, eager "
                                "and replayed steps) and candidate pairs at the end; the collision kernels "
                                "are timed inside value, not in the roofline of the step kernel")
    out["roofline"]["copy_probe"] = copy_probe()
    if not args.no_cache_leg and args.workload != "random_block_100":
        log("cache-resident leg: random_block_100, FP32 and FP64")
        w2 = build_workload("random_block_100")
        r2 = time_gpu(w2, 32, kernel, args.steps, args.warmup, autotune, graph=use_graph)
        r2d = time_gpu(w2, 64, kernel, args.steps, args.warmup, autotune, graph=use_graph)
        out["cache_resident"] = {"f32": lattice_leg(w2, 32, r2, args.steps, args.kernel),
                                 "f64": lattice_leg(w2, 64, r2d, args.steps, args.kernel),
                                 "note": "state of 52 MB (FP32) or 104 MB (FP64) per buffer: both ping-pong "
                                         "buffers fit the 256 MB last-level cache, so the HBM fraction is "
                                         "not an HBM measurement"}
        if not args.no_cpu:
            log("cpu baseline of the 100^3 block (oracle)")
            out["cache_resident"]["cpu_baseline"] = cpu_baseline(w2, budget_s=8.0)
        del w2
    if not args.no_batch_leg:
        log("batched leg: %d objects, %d steps" % (args.batch_objects, args.batch_steps))
        out["batched"] = time_batch(args.batch_objects, args.batch_steps, args.one_by_one_sample)
    if not args.no_collision_leg:
        log("collision-scheme leg: clapper, 512 pairs of colliding bodies")
        out["collision_schemes"] = time_collision_schemes(graph=not args.eager)
        import workloads
        wb, _ = workloads.colliding_bodies(pairs=(8, 8, 8), steps=2000)
        out["collision_schemes_bodies"] = time_collision_schemes(2000, graph=not args.eager, w=wb)
        del wb
    if not args.no_adjoint_leg:
        log("adjoint leg: design lattice, %d steps" % args.adjoint_steps)
        out["adjoint"] = time_adjoint(args.adjoint_steps)
        if args.adjoint_contact_steps > 0:
            log("adjoint leg through contact: colliding bodies, %d steps" % args.adjoint_contact_steps)
            try:
                out["adjoint_contact"] = time_adjoint_contact(args.adjoint_contact_steps)
            except Exception as e:   # reported, so that the other legs still print
                out["adjoint_contact"] = {"error": "%s: %s" % (type(e).__name__, e)}
    if not args.no_paper_shape_leg:
        log("paper-shape leg: cubes 8^3 .. 40^3")
        out["paper_shape"] = time_paper_shape()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        crop = args.cpu_crop if w["params"].get("self_collision_on") else None
        out["cpu_baseline"] = cpu_baseline(w, crop=crop)
        if "batched" in out:
            log("cpu baseline of the batched objects (oracle, all host cores)")
            cb = cpu_batch_baseline(args.batch_objects)
            out["batched"]["cpu_baseline"] = cb
            out["batched"]["speedup_vs_cpu"] = out["batched"]["value"] / cb["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
