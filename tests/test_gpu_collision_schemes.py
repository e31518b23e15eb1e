"""Self-collision schemes (section "Speedup of self collision schemes",
Table 3) on the GPU: the clapper stepped with candidates from all voxels or
the surface only, rebuilt every step or by the horizon rule.  The schemes
change the cost, not the forces: all four trajectories are identical, and
each rebuild rule equals the oracle run with the same rule."""
import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import workloads
from parity import build_gpu, build_oracle

pytestmark = pytest.mark.gpu

STEPS = 3000


def gpu_run(w, all_voxels, every_step, steps=STEPS):
    s = vx.Sim(w["grid"], w["materials"], precision=64, **w["params"])
    s.set_collision_mode(all_voxels, every_step)
    s.set_fixed(w["fixed"])
    s.step(steps)
    c = s.counters()
    return s.read_state(), c


def interior_mask(grid):
    g = grid > 0
    inner = g.copy()
    for ax in range(3):
        for sh in (1, -1):
            nb = np.roll(g, sh, axis=ax)
            edge = [slice(None)] * 3
            edge[ax] = 0 if sh == 1 else -1
            nb[tuple(edge)] = False
            inner &= nb
    return inner.reshape(-1)


def test_rebuild_rules_give_identical_trajectories_and_match_oracle():
    w = workloads.clapper()
    runs = {}
    for all_voxels in (0, 1):
        for every in (0, 1):
            print("[case] clapper all=%d every=%d" % (all_voxels, every), flush=True)
            runs[(all_voxels, every)] = gpu_run(w, all_voxels, every)
    # the rebuild rule changes when the lists are rebuilt, never the forces
    for all_voxels in (0, 1):
        a, b = runs[(all_voxels, 0)][0], runs[(all_voxels, 1)][0]
        for k in ("u", "q", "v", "w"):
            assert np.array_equal(a[k], b[k]), (all_voxels, k)
    # every-step schemes rebuild before each step; the horizon rule far less
    assert runs[(0, 1)][1]["rebuilds"] >= STEPS
    assert runs[(0, 0)][1]["rebuilds"] < STEPS // 3
    for every in (0, 1):
        o = build_oracle(w)
        if every:
            o.set_rebuild_every_step(True)
        assert o.step(STEPS) == 0
        uo = o.read_state()["u"]
        ug = runs[(0, every)][0]["u"]
        assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()


def test_all_voxels_mode_is_fixed_at_bind():
    w = workloads.clapper()
    s = vx.Sim(w["grid"], w["materials"], precision=32, **w["params"])
    s.set_collision_mode(True, False)
    s.bind()
    s.set_collision_mode(True, True)     # the rebuild rule may change
    with pytest.raises(vx.VoxsimError):
        s.set_collision_mode(False, True)


def test_all_voxels_equals_surface_until_an_interior_voxel_is_a_candidate():
    """With all voxels in the search, the four interior voxels of the base
    (under the arms) join the lists once the arms' contracting inner layers
    bring arm voxels within the horizon; until then the two searches give
    the same forces and the same trajectory."""
    w = workloads.clapper()
    inner = interior_mask(w["grid"])
    assert inner.sum() == 4
    sims = []
    for all_voxels in (0, 1):
        s = vx.Sim(w["grid"], w["materials"], precision=64, **w["params"])
        s.set_collision_mode(all_voxels, 0)
        s.set_fixed(w["fixed"])
        sims.append(s)
    first_inner = None
    for k in range(1, 13):
        for s in sims:
            s.step(250)
        a, b = sims[1].candidates(), sims[0].candidates()
        if any(inner[i] or inner[j] for i, j in a):
            first_inner = k * 250
            break
        sa, sb = sims[0].read_state(), sims[1].read_state()
        for key in ("u", "q", "v", "w"):
            assert np.array_equal(sa[key], sb[key]), (k * 250, key)
        assert a == b, k * 250
    print("[case] first interior candidate within step", first_inner, flush=True)



def test_candidate_lists_do_not_depend_on_the_cap():
    """Each voxel's list is built in LDS sized by the cap and sorted by
    rank: with 100 slots the clapper's lists, pair count, rebuild count and
    trajectory (every-step rebuilds, 1500 FP64 steps) are bitwise those of
    the default 32 slots, none of which overflows."""
    w = workloads.clapper()
    out = []
    for cap in (32, 100):
        params = dict(w["params"], contact_cap=cap)
        s = vx.Sim(w["grid"], w["materials"], precision=64, **params)
        s.set_collision_mode(False, True)
        s.set_fixed(w["fixed"])
        s.step(1500)
        out.append((s.read_state(), s.counters(), s.candidates()))
    (sa, ca, la), (sb, cb, lb) = out
    assert ca["rebuilds"] == cb["rebuilds"] and ca["pairs"] == cb["pairs"] and ca["pairs"] > 0, (ca, cb)
    assert la == lb
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(sa[k], sb[k]), k
