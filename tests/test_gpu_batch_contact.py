"""Contact between the objects of a batch (Introduction: collisions "allow
multiple bodies to interact"; section Self collision detection and
handling): 48 free bodies of 3^3 to 5^3 voxels in approaching pairs, each
its own object of one batch placed by its world origin, against the FP64
oracle run on one lattice that holds the same bodies.  Bodies lie more
than 3 cells apart in lattice Manhattan distance, so the oracle's lattice
exclusion and the batch's per-object exclusion select the same pairs; the
batch sums a voxel's contact forces in object order, the oracle in lattice
order, so the two agree to rounding."""
import numpy as np
import pytest

import paper_1212_2845_amd as vx
import workloads
from parity import build_oracle, compare

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def announce(msg):
    print("[case] " + msg, flush=True)


def body_objects(w, bodies):
    """Each body's block of the lattice as an object: its grid, world
    origin, the lattice cells of its cells in object order, and its
    initial state."""
    grid = w["grid"]
    nz, ny, nx = grid.shape
    l = w["params"]["voxel_size"]
    o = w["params"]["origin"]
    out = []
    for (x0, y0, z0, sx, sy, sz) in bodies:
        g = np.ascontiguousarray(grid[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx])
        zz, yy, xx = np.meshgrid(np.arange(z0, z0 + sz), np.arange(y0, y0 + sy), np.arange(x0, x0 + sx),
                                 indexing="ij")
        cells = ((zz * ny + yy) * nx + xx).reshape(-1)
        st = {k: w["state"][k][cells] for k in ("u", "q", "v", "w")}
        out.append({"grid": g, "origin": (o[0] + x0 * l, o[1] + y0 * l, o[2] + z0 * l), "cells": cells, "state": st})
    return out


_REF = {}


def _reference():
    if not _REF:
        w, bodies = workloads.colliding_bodies()
        o = build_oracle(w)
        assert o.step(600) == 0
        _REF["mid"] = (sorted(o.candidates()), o.rebuilds)
        assert o.step(400) == 0
        _REF["end"] = (sorted(o.candidates()), o.rebuilds, o.read_state())
        _REF["w"], _REF["objs"] = w, body_objects(w, bodies)
    return _REF


def make_batch(r, precision):
    w, objs = r["w"], r["objs"]
    b = vx.Batch([ob["grid"] for ob in objs], w["materials"], precision=precision,
                 origins=[ob["origin"] for ob in objs], **w["params"])
    b.bind()
    for i, ob in enumerate(objs):
        b.write_state(i, **ob["state"])
    return b


def lattice_pairs(b, objs):
    """The batch's candidate pairs as sorted (lattice cell, lattice cell)."""
    out = []
    for (oa, ca), (ob_, cb) in b.candidates():
        a, c = int(objs[oa]["cells"][ca]), int(objs[ob_]["cells"][cb])
        out.append((min(a, c), max(a, c)))
    return sorted(out)


def gathered(b, objs, ncell):
    """The batch's state scattered back to lattice cells."""
    st = {"u": np.zeros((ncell, 3)), "q": np.tile([1.0, 0, 0, 0], (ncell, 1)), "v": np.zeros((ncell, 3)),
          "w": np.zeros((ncell, 3))}
    for i, ob in enumerate(objs):
        s = b.read_state(i)
        for k in st:
            st[k][ob["cells"]] = s[k]
    return st


def test_batch_contact_equals_one_lattice_fp64():
    r = _reference()
    w, objs = r["w"], r["objs"]
    announce("batch contact 48 bodies fp64")
    b = make_batch(r, 64)
    assert b.counters()["objects"] == 48
    assert b.contact_counters()["surface"] >= 1000
    f = w["grid"].reshape(-1) > 0
    b.step(600)
    cand_mid, reb_mid = r["mid"]
    assert len(cand_mid) >= 100
    assert lattice_pairs(b, objs) == cand_mid
    assert b.contact_counters()["rebuilds"] == reb_mid
    b.step(400)
    cand_end, reb_end, ref = r["end"]
    assert lattice_pairs(b, objs) == cand_end
    assert b.contact_counters()["rebuilds"] == reb_end
    e = compare(gathered(b, objs, w["grid"].size), ref, f)
    print(e, len(cand_mid), len(cand_end), reb_end, flush=True)
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12, e


def test_batch_contact_fp32_max_displacement():
    r = _reference()
    w, objs = r["w"], r["objs"]
    announce("batch contact 48 bodies fp32")
    b = make_batch(r, 32)
    b.step(1000)
    f = w["grid"].reshape(-1) > 0
    got = gathered(b, objs, w["grid"].size)
    ug = np.linalg.norm(got["u"][f], axis=1).max()
    uo = np.linalg.norm(r["end"][2]["u"][f], axis=1).max()
    assert abs(ug / uo - 1.0) < 1e-4, (ug, uo)


def test_batch_without_contact_lets_bodies_pass_through():
    """The same batch with contact off: the bodies never touch, each moves
    as it would alone, so every object keeps its kinetic energy up to its
    bond damping of the spin-up, and the pairs overlap."""
    r = _reference()
    w, objs = r["w"], r["objs"]
    params = dict(w["params"], self_collision_on=0)
    announce("batch without contact")
    b = vx.Batch([ob["grid"] for ob in objs], w["materials"], precision=64,
                 origins=[ob["origin"] for ob in objs], **params)
    b.bind()
    for i, ob in enumerate(objs):
        b.write_state(i, **ob["state"])
    b.step(1000)
    # the first pair's facing faces have crossed: body a's largest x
    # position is beyond body b's smallest
    l = w["params"]["voxel_size"]
    pos = []
    for i in (0, 1):
        g = objs[i]["grid"]
        x, _, _ = workloads.cell_coords(g.shape)
        s = b.read_state(i)
        pos.append(objs[i]["origin"][0] + (x + 0.5) * l + s["u"][:, 0])
    assert pos[0].max() > pos[1].min()
