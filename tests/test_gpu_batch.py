"""Batched persistent stepping: many independent objects in one launch.

Each object of a batch must evolve as it does alone: against the
single-lattice fused path (same device arithmetic; different tiles, so equal
to rounding) and against the FP64 oracle.
"""
import numpy as np
import pytest

import paper_1212_2845_amd as vx
import workloads
from parity import build_oracle, compare, perturbed_state

pytestmark = pytest.mark.gpu

MATS = [workloads.EMPTY, workloads._mat(1e6), workloads._mat(1e8), workloads._mat(1e6, cte=0.01),
        workloads._mat(1e6, cte=-0.01)]
PARAMS = dict(gravity=9.81, zeta_bond=0.5, zeta_col=0.5, floor_on=1, temp_amp=20.0, temp_freq=200.0)


def announce(msg):
    print("[case] " + msg, flush=True)


def make_objects(n, seed, lo=3, hi=12, perturb=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    grids, states = [], []
    for i in range(n):
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        g = rng.integers(0, 5, size=(nz, ny, nx)).astype(np.uint8)
        if i % 4 == 0:
            g[g == 2] = 1               # some objects without the stiff material: a larger dt
        grids.append(g)
        states.append(perturbed_state(g.size, seed + 100 + i, 1e-6, 1e-3, 0.5, 1e-3) if perturb else None)
    return grids, states


def run_batch(grids, states, steps, precision, **kw):
    b = vx.Batch(grids, MATS, precision=precision, **PARAMS)
    b.bind()
    for k, v in kw.items():
        if k == "launch":
            b.set_launch(*v)
    for i, st in enumerate(states):
        if st is not None:
            b.write_state(i, **st)
    b.step(steps)
    return b


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 2e-5)])
def test_batch_matches_single_objects(precision, tol):
    grids, states = make_objects(12, seed=11)
    announce("batch of 12 vs single p=%d" % precision)
    b = run_batch(grids, states, 150, precision)
    for i, g in enumerate(grids):
        s = vx.Sim(g, MATS, precision=precision, **PARAMS)
        s.write_state(**states[i])
        assert abs(s.dt / b.dt(i) - 1.0) < 1e-15
        s.step(150)
        e = compare(b.read_state(i), s.read_state(), g.reshape(-1) > 0)
        assert max(e["u"], e["v"], e["w"]) < tol and e["q"] < tol, (i, e)


def test_batch_thin_objects_match_single_objects():
    """Objects one or two cells thick and long in y, and one longer than a
    tile in x: the batch kernel's tile (at most 64 x 64 cells, 256 in all)
    covers each, FP64 equal to the single-lattice path to rounding."""
    rng = np.random.Generator(np.random.PCG64(51))
    shapes = [(3, 100, 1), (4, 150, 2), (3, 1, 70), (2, 70, 3), (5, 5, 5)]
    grids = [rng.integers(1, 5, size=sh).astype(np.uint8) for sh in shapes]
    states = [perturbed_state(g.size, 60 + i, 1e-6, 1e-3, 0.5, 1e-3) for i, g in enumerate(grids)]
    announce("batch of thin objects")
    b = run_batch(grids, states, 100, 64)
    for i, g in enumerate(grids):
        s = vx.Sim(g, MATS, precision=64, **PARAMS)
        s.write_state(**states[i])
        s.step(100)
        e = compare(b.read_state(i), s.read_state(), g.reshape(-1) > 0)
        assert max(e["u"], e["v"], e["w"]) < 1e-12 and e["q"] < 1e-12, (i, shapes[i], e)


def test_batch_matches_oracle_fp64():
    grids, states = make_objects(4, seed=21, lo=3, hi=7)
    announce("batch vs oracle")
    b = run_batch(grids, states, 200, 64)
    for i, g in enumerate(grids):
        w = workloads._workload(g, MATS, workloads._base_params(**PARAMS), 200)
        w["state"] = states[i]
        o = build_oracle(w)
        assert abs(o.dt / b.dt(i) - 1.0) < 1e-15
        assert o.step(200) == 0
        e = compare(b.read_state(i), o.read_state(), g.reshape(-1) > 0)
        assert max(e["u"], e["v"], e["w"]) < 1e-10 and e["q"] < 1e-12, (i, e)


def test_batch_launch_split_is_bitwise():
    """Splitting the steps over several launches, or changing the number of
    workgroups, runs the same arithmetic per object."""
    grids, states = make_objects(10, seed=31)
    announce("batch launch split")
    ref = run_batch(grids, states, 60, 32)
    alt = run_batch(grids, states, 60, 32, launch=(3, 7))
    for i in range(len(grids)):
        a, r = alt.read_state(i), ref.read_state(i)
        for k in ("u", "q", "v", "w"):
            assert np.array_equal(a[k], r[k]), (i, k)


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 2e-5)])
def test_tile_rules_match_single_objects(precision, tol):
    """Footprints wider than one 64-cell tile, where the evened-width rule
    cuts them otherwise than the widest-rows rule, and narrower ones: under
    either rule each object equals the single-lattice path to rounding, and
    the two rules agree."""
    rng = np.random.Generator(np.random.PCG64(71))
    shapes = [(70, 3, 2), (100, 5, 2), (130, 4, 2), (66, 12, 2), (33, 30, 4), (9, 40, 2)]
    grids = [rng.integers(0, 5, size=(nz, ny, nx)).astype(np.uint8) for nx, ny, nz in shapes]
    states = [perturbed_state(g.size, 80 + i, 1e-6, 1e-3, 0.5, 1e-3) for i, g in enumerate(grids)]
    announce("tile rules p=%d" % precision)
    runs = []
    for rule in (0, 1):
        b = vx.Batch(grids, MATS, precision=precision, **PARAMS)
        b.set_tile_rule(rule)
        b.bind()
        for i, st in enumerate(states):
            b.write_state(i, **st)
        b.step(120)
        runs.append(b)
    differ = sum(runs[0].tile(i)[1:] != runs[1].tile(i)[1:] for i in range(len(grids)))
    assert differ >= 4
    for i, g in enumerate(grids):
        s = vx.Sim(g, MATS, precision=precision, **PARAMS)
        s.write_state(**states[i])
        s.step(120)
        want = s.read_state()
        filled = g.reshape(-1) > 0
        for b in runs:
            e = compare(b.read_state(i), want, filled)
            assert max(e["u"], e["v"], e["w"]) < tol and e["q"] < tol, (i, b.tile(i), e)
        e = compare(runs[1].read_state(i), runs[0].read_state(i), filled)
        assert max(e["u"], e["v"], e["w"]) < tol and e["q"] < tol, (i, e)


def test_batch_autotune_restores_state():
    grids, states = make_objects(16, seed=41)
    announce("batch autotune")
    b = vx.Batch(grids, MATS, precision=32, **PARAMS)
    b.bind()
    for i, st in enumerate(states):
        b.write_state(i, **st)
    before = [b.read_state(i) for i in range(len(grids))]
    nw = b.autotune(steps=5)
    assert 1 <= nw <= len(grids)
    assert b.tile(0)[0] in (0, 1)
    assert b.counters()["steps"] == 0
    for i in range(len(grids)):
        now = b.read_state(i)
        for k in ("u", "q", "v", "w"):
            assert np.array_equal(now[k], before[i][k])


def test_batch_of_generated_objects_runs():
    """A slice of the 4096-object workload (8^3 .. 32^3, five classes) on the
    floor: finite, and the bottom layers rest on the floor."""
    objs = workloads.batch_objects(count=64, seed=4, steps=200)
    announce("batch of 64 generated objects")
    b = vx.Batch([o["grid"] for o in objs], objs[0]["materials"], precision=32, **objs[0]["params"])
    b.step(200)
    for i in (0, 17, 63):
        st = b.read_state(i)
        assert np.isfinite(st["u"]).all() and np.isfinite(st["v"]).all()


@pytest.mark.parametrize("collide", [0, 1])
def test_graph_captured_steps_replay_like_eager(collide):
    """vx_step_enqueue recorded by stream capture into a HIP graph replays
    the recorded steps exactly as eager stepping runs them, replay after
    replay, with eager host work (state writes, status checks) between."""
    import torch
    w = workloads._workload(np.ones((6, 5, 7), np.uint8), MATS[:3],
                            workloads._base_params(**dict(PARAMS, self_collision_on=collide)), 12)
    st0 = perturbed_state(w["grid"].size, 77, 1e-6, 1e-3, 0.5, 1e-3)
    announce("graph capture collide=%d" % collide)
    ref = vx.from_workload(w, precision=32)
    ref.write_state(**st0)
    ref.step(12)
    want = ref.read_state()
    side = torch.cuda.Stream()
    s = vx.from_workload(w, precision=32, stream=side.cuda_stream)
    s.bind()
    s.write_state(**st0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.step_enqueue(12)
    for rep in range(3):
        s.write_state(**st0)
        g.replay()
        torch.cuda.synchronize()
        s.status()
        got = s.read_state()
        for k in ("u", "q", "v", "w"):
            assert np.array_equal(got[k], want[k]), (rep, k)


def test_full_size_batch_sampled_against_oracle():
    """The 4096-object batch of the benchmark (bounding boxes U{8..32}^3,
    about 26M voxels, FP32) in the launch configuration bench.py times
    (autotuned workgroup count, one persistent launch for all steps).  Four
    objects (the largest, the smallest and two at random) start from a
    perturbed state, the rest at rest on the floor; after 100 steps each of
    the four equals the FP64 oracle run on that object alone, to the FP32
    bar (largest displacement within 1e-4 relative)."""
    objs = workloads.batch_objects(count=4096, seed=4, steps=100)
    announce("full size batch 4096")
    b = vx.Batch([o["grid"] for o in objs], objs[0]["materials"], precision=32, **objs[0]["params"])
    b.bind()
    b.autotune(steps=20)
    sizes = np.array([int((o["grid"] > 0).sum()) for o in objs])
    rng = np.random.Generator(np.random.PCG64(41))
    picks = [int(sizes.argmax()), int(sizes.argmin())] + rng.choice(len(objs), 2, replace=False).tolist()
    starts = {}
    for i in picks:
        starts[i] = perturbed_state(objs[i]["grid"].size, 300 + i, 1e-6, 1e-3, 0.5, 1e-3)
        b.write_state(i, **starts[i])
        starts[i] = b.read_state(i)      # the FP32-rounded input the oracle starts from
    b.step(100)
    for i in picks:
        w = dict(objs[i])
        w["state"] = starts[i]
        o = build_oracle(w)
        assert abs(o.dt / b.dt(i) - 1.0) < 1e-15
        assert o.step(100) == 0
        got, ref = b.read_state(i), o.read_state()
        filled = objs[i]["grid"].reshape(-1) > 0
        ug = np.linalg.norm(got["u"][filled], axis=1).max()
        uo = np.linalg.norm(ref["u"][filled], axis=1).max()
        e = compare(got, ref, filled)
        assert abs(ug / uo - 1.0) < 1e-4 and e["u"] < 1e-3, (i, sizes[i], ug, uo, e)


def test_autotune_failure_restores_batch():
    """A trial run that goes unstable (bond damping far above 1) makes the
    autotuner return VX_EUNSTABLE with the state, the step count, the
    status flags and the tile rule as they were before the call."""
    g = np.ones((6, 6, 6), np.uint8)
    grids = [g, g]
    announce("batch autotune failure")
    b = vx.Batch(grids, [workloads.EMPTY, workloads._mat(1e6)], precision=64,
                 **workloads._base_params(zeta_bond=3.0))
    b.bind()
    for i in range(2):
        st = perturbed_state(g.size, 310 + i, 1e-7, 1e-4, 0.0, 0.0)
        b.write_state(i, u=st["u"], v=st["v"])
    before = [b.read_state(i) for i in range(2)]
    b.set_tile_rule(1)
    with pytest.raises(vx.VoxsimError) as e:
        b.autotune(steps=3000)
    assert e.value.code == vx.VX_EUNSTABLE
    assert b.tile(0)[0] == 1
    assert b.counters()["steps"] == 0
    for i in range(2):
        after = b.read_state(i)
        for k in ("u", "q", "v", "w"):
            assert np.array_equal(after[k], before[i][k]), (i, k)
    b.step(1)          # the sticky status flag was restored too: one step is fine
