"""Parity of the HIP step (through the C ABI) with the FP64 oracle.

Bars: FP64 state within 1e-10 of the oracle (displacement error over the
largest displacement; velocities likewise over their largest magnitude), FP32
largest displacement within 1e-4, bitwise equality run to run, and the
split and fused kernels (same device functions) equal to rounding.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import workloads
from parity import build_gpu, build_oracle, compare, perturbed_state

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_MAXDISP_TOL = 1e-4
KERNELS = [vx.KERNEL_SPLIT, vx.KERNEL_FUSED]


def announce(msg):
    print("[case] " + msg, flush=True)


def run_pair(w, steps, precision=64, kernel=vx.KERNEL_FUSED):
    g = build_gpu(w, precision=precision, kernel=kernel)
    o = build_oracle(w)
    g.step(steps)
    assert o.step(steps) == 0
    return g, o


def filled_of(w):
    return w["grid"].reshape(-1) > 0


def hetero_block(shape=(5, 6, 7), seed=41, fill=0.85, act=True):
    mats = workloads.random_materials(3, seed=seed, cte_max=0.01)
    g = workloads.random_grid(shape, 3, fill, seed + 1)
    w = workloads._workload(g, mats, workloads._base_params(zeta_bond=0.3, zeta_slow=0.01,
                                                            temp_amp=15.0, temp_freq=200.0),
                            300, name="hetero_%dx%dx%d" % shape)
    n = g.size
    w["state"] = perturbed_state(n, seed + 2, u_scale=2e-6, v_scale=2e-3, w_scale=1.0, rot_scale=2e-3)
    if act:
        rng = np.random.Generator(np.random.PCG64(seed + 3))
        w["amp"] = rng.uniform(5.0, 20.0, n)
        w["phase"] = rng.uniform(0.0, 2 * math.pi, n)
    return w


def test_cantilever_c1_full_run_fp64():
    """C1 as specified: 10,000 steps FP64 (fused kernel); displacement,
    orientation, tip deflection and the elastic and gravitational energies
    of the final state equal the oracle's.  (By then the beam has settled:
    velocities are ~1e-7 of their peak, so they are compared in the
    1000-step test above rather than relative to their own final size.)"""
    w = workloads.cantilever(steps=10000)
    announce("cantilever_20x4x4 fp64 10000 steps")
    g, o = run_pair(w, 10000, 64, vx.KERNEL_FUSED)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    assert e["u"] < FP64_TOL and e["q"] < 1e-12, e
    x, _, _ = workloads.cell_coords(w["grid"].shape)
    ug, uo = g.read_state()["u"], o.read_state()["u"]
    assert abs(ug[x == 19, 2].mean() / uo[x == 19, 2].mean() - 1) < 1e-10
    eg, eo = g.energy(), o.energy()
    for kg, ko in (("elastic", "elastic"), ("gravity", "gravity")):
        assert abs(eg[kg] - eo[ko]) <= 1e-8 * max(abs(eo[ko]), 1e-300), (kg, eg[kg], eo[ko])


@pytest.mark.parametrize("kernel", KERNELS)
def test_cantilever_fp64(kernel):
    w = workloads.cantilever(steps=1000)
    announce("cantilever_20x4x4 fp64 kernel=%d 1000 steps" % kernel)
    g, o = run_pair(w, 1000, 64, kernel)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    print(e, flush=True)
    assert e["u"] < FP64_TOL and e["v"] < FP64_TOL and e["w"] < FP64_TOL and e["q"] < 1e-12


@pytest.mark.parametrize("kernel", KERNELS)
def test_hetero_block_fp64(kernel):
    """Several materials, empty cells, perturbed rotations, per-voxel
    actuation: every bond orientation and branch of the bond math."""
    w = hetero_block()
    announce("hetero block fp64 kernel=%d" % kernel)
    g, o = run_pair(w, 300, 64, kernel)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    print(e, flush=True)
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12


@pytest.mark.parametrize("kernel", KERNELS)
def test_impact_on_floor_fp64(kernel):
    """Reduced impact case: random soft/stiff block hitting the floor at the
    speed of a 5 mm drop, friction on."""
    w = workloads.random_block(n=10, seed=2, impact=True)
    announce("impact 10^3 fp64 kernel=%d" % kernel)
    g, o = run_pair(w, 400, 64, kernel)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    print(e, flush=True)
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL
    assert np.array_equal(g.read_flags()["static"], o.read_flags()["static"])


def test_two_cubes_collision_fp64():
    n, gap = 3, 1
    nx = 2 * n + gap
    grid = np.zeros((n, n, nx), np.uint8)
    grid[:, :, :n] = 1
    grid[:, :, n + gap:] = 1
    x, _, _ = workloads.cell_coords(grid.shape)
    v = np.zeros((grid.size, 3))
    v[x < n, 0] = 2.0
    v[x >= n + gap, 0] = -2.0
    w = workloads._workload(grid, [workloads.EMPTY, workloads._mat(1e6)],
                            workloads._base_params(zeta_bond=0.5, zeta_col=0.5, self_collision_on=1),
                            600, velocity=v, name="two_cubes")
    announce("two cubes collision fp64")
    g, o = run_pair(w, 600, 64)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    print(e, g.counters(), o.rebuilds, flush=True)
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL
    assert g.candidates() == o.candidates()
    assert g.counters()["rebuilds"] == o.rebuilds


@pytest.mark.parametrize("kernel", KERNELS)
def test_cantilever_fp32_max_displacement(kernel):
    w = workloads.cantilever(steps=1000)
    announce("cantilever fp32 kernel=%d" % kernel)
    g, o = run_pair(w, 1000, 32, kernel)
    ug = np.linalg.norm(g.read_state()["u"], axis=1).max()
    uo = np.linalg.norm(o.read_state()["u"], axis=1).max()
    print(ug, uo, abs(ug / uo - 1), flush=True)
    assert abs(ug / uo - 1.0) < FP32_MAXDISP_TOL


@pytest.mark.parametrize("kernel", KERNELS)
def test_hetero_block_fp32(kernel):
    w = hetero_block(seed=51)
    announce("hetero block fp32 kernel=%d" % kernel)
    g, o = run_pair(w, 300, 32, kernel)
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    print(e, flush=True)
    ug = np.linalg.norm(g.read_state()["u"], axis=1).max()
    uo = np.linalg.norm(o.read_state()["u"], axis=1).max()
    assert abs(ug / uo - 1.0) < FP32_MAXDISP_TOL
    assert e["u"] < 1e-3


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 2), (3, 1, 1), (1, 4, 1), (2, 3, 67), (5, 33, 17)])
def test_edge_shapes_fp64(shape):
    """Single voxel (no bonds: free fall), single bonds along each axis,
    thin and ragged lattices that leave partial tiles."""
    mats = workloads.random_materials(2, seed=61)
    g = workloads.random_grid(shape, 2, 0.9 if np.prod(shape) > 4 else 1.0, seed=62)
    w = workloads._workload(g, mats, workloads._base_params(gravity=9.81, zeta_bond=0.2), 200)
    w["state"] = perturbed_state(g.size, 63, 1e-6, 1e-3, 0.5, 1e-3)
    announce("edge shape %s" % (shape,))
    for kernel in KERNELS:
        gs, o = run_pair(w, 200, 64, kernel)
        e = compare(gs.read_state(), o.read_state(), filled_of(w))
        assert max(e["u"], e["v"], e["w"]) < FP64_TOL, (kernel, e)


@pytest.mark.parametrize("shape_id", range(len(vx.FUSED_SHAPES)))
@pytest.mark.parametrize("zc", [1, 3, 0])
def test_fused_tiles_fp64(shape_id, zc):
    """Every fused tile shape and z-chunk (odd chunk lengths, chunk of one
    slab, default) on a ragged lattice that leaves partial tiles in x and y
    and a partial last chunk in z."""
    w = hetero_block(shape=(7, 13, 53), seed=91)
    announce("fused tile %s zc=%d" % (vx.FUSED_SHAPES[shape_id], zc))
    g = build_gpu(w, 64, vx.KERNEL_FUSED)
    g.set_fused_tile(shape_id, zc)
    o = build_oracle(w)
    g.step(60)
    assert o.step(60) == 0
    e = compare(g.read_state(), o.read_state(), filled_of(w))
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12, e


def test_autotune_keeps_state():
    """Autotuning times launches from the current state without advancing it."""
    w = hetero_block(shape=(9, 10, 11), seed=95)
    announce("autotune")
    g = build_gpu(w, 32, vx.KERNEL_FUSED)
    g.step(10)
    before = g.read_state()
    t0 = g.time
    cfg = g.autotune(iters=2)
    assert 0 <= cfg["shape"] < len(vx.FUSED_SHAPES) and cfg["zc"] >= 1
    after = g.read_state()
    assert g.time == t0
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(before[k], after[k])
    # same tiles as g: the heuristic tile for 10 steps, the tuned one after
    ref = build_gpu(w, 32, vx.KERNEL_FUSED)
    ref.step(10)
    ref.set_fused_tile(cfg["shape"], cfg["zc"])
    ref.step(10)
    g.step(10)
    e = compare(g.read_state(), ref.read_state(), filled_of(w))
    assert e["u"] == 0.0 and e["q"] == 0.0


def test_empty_lattice_steps():
    g = np.zeros((3, 3, 3), np.uint8)
    s = vx.Sim(g, [workloads.EMPTY, workloads._mat(1e6)])
    announce("empty lattice")
    s.step(5)
    assert s.counters()["voxels"] == 0


@pytest.mark.parametrize("precision", [32, 64])
def test_deterministic_and_split_matches_fused(precision):
    """Run-to-run bitwise equality of the fused kernel; the split path runs
    the same device functions but the compiler may contract them into FMAs
    differently, so it agrees to rounding (FP64 1e-12, FP32 1e-5 of the
    largest displacement)."""
    w = hetero_block(shape=(9, 10, 11), seed=71)
    announce("determinism p=%d" % precision)
    states = []
    for kernel in (vx.KERNEL_FUSED, vx.KERNEL_FUSED, vx.KERNEL_SPLIT):
        s = build_gpu(w, precision, kernel)
        s.step(100)
        states.append(s.read_state())
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(states[0][k], states[1][k])
    filled = filled_of(w)
    e = compare(states[2], states[0], filled)
    tol = 1e-12 if precision == 64 else 1e-5
    assert e["u"] < tol and e["q"] < tol, e


def test_unstable_reports_error():
    """Bond damping far above 1 is unstable (the paper warns of values
    above 1): the step reports VX_EUNSTABLE instead of running on."""
    g = np.ones((6, 6, 6), np.uint8)
    s = vx.Sim(g, [workloads.EMPTY, workloads._mat(1e6)], zeta_bond=3.0)
    st = perturbed_state(g.size, 81, 1e-7, 1e-4, 0.0, 0.0)
    s.write_state(u=st["u"], v=st["v"])
    announce("unstable")
    rc = s.step_rc(3000)
    assert rc == vx.VX_EUNSTABLE


def _neighbourhood_oracle(w, state, cell, nx, ny, nz, dt):
    """Oracle on the 3x3x3 block around `cell` (cells outside the lattice
    empty), with the same materials, parameters, state and timestep dt (the
    block alone would pick its own stable step from fewer material pairs);
    returns the oracle's state of the centre after one step."""
    x, y, z = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    sub = np.zeros((3, 3, 3), np.uint8)
    idx = np.full((3, 3, 3), -1, np.int64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if abs(dx) + abs(dy) + abs(dz) > 1:
                    continue            # only the face neighbours act on the centre
                X, Y, Z = x + dx, y + dy, z + dz
                if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz:
                    c = X + nx * (Y + ny * Z)
                    sub[dz + 1, dy + 1, dx + 1] = w["grid"].reshape(-1)[c]
                    idx[dz + 1, dy + 1, dx + 1] = c
    params = dict(w["params"])
    o = params.get("origin", (0.0, 0.0, 0.0))
    l = params["voxel_size"]
    params["origin"] = (o[0] + (x - 1) * l, o[1] + (y - 1) * l, o[2] + (z - 1) * l)
    params["self_collision_on"] = 0
    params["dt_scale"] = 1.0
    dt_own = oracle.Sim(sub, w["materials"], **params).dt
    params["dt_scale"] = dt / dt_own
    assert params["dt_scale"] <= 1.0
    orc = oracle.Sim(sub, w["materials"], **params)
    assert abs(orc.dt / dt - 1.0) < 1e-15
    sel = idx.reshape(-1)
    st = {}
    for k, d in (("u", 3), ("q", 4), ("v", 3), ("w", 3)):
        a = np.zeros((27, d))
        if k == "q":
            a[:, 0] = 1.0
        a[sel >= 0] = state[k][sel[sel >= 0]]
        st[k] = a
    orc.write_state(**st)
    assert orc.step(1) == 0
    r = orc.read_state()
    return {k: r[k][13] for k in r}


# One FP32 step from a perturbed state (rotations of 1e-3 rad on 1 mm
# voxels), error over the larger of the oracle's value and the start value,
# per quantity.  The velocity bar is the loosest: the step's change of
# velocity (up to eight times the start velocity) is the net of bond forces
# whose rotational and translational parts nearly cancel, so FP32 rounding
# of the terms shows up amplified in the net (measured on the samples:
# u 5.7e-6, v 2.3e-5, w 5.5e-7, q 8.7e-8).
FP32_ONE_STEP = {"u": 2e-5, "v": 5e-5, "w": 2e-6, "q": 5e-7}
FP64_ONE_STEP = {"u": 1e-10, "v": 1e-10, "w": 1e-10, "q": 1e-10}


@pytest.mark.parametrize("precision", [64, 32])
def test_full_size_blob_lattice_sampled(precision):
    """256^3 lattice of the HBM-resident benchmark, in the launch
    configuration bench.py times (fused kernel, autotuned tile): one step
    from a perturbed state, then 48 sampled voxels (interior, faces, edges,
    corners) recomputed one by one by the oracle on their neighbourhood."""
    tols = FP64_ONE_STEP if precision == 64 else FP32_ONE_STEP
    n = 256
    w = workloads.blob_lattice(n=n, seed=3)
    w["params"]["temp_phase"] = 0.7      # non-zero temperature at t = 0
    ncell = n ** 3
    announce("full size 256^3 p=%d" % precision)
    st = perturbed_state(ncell, 97, 1e-6, 1e-3, 0.5, 1e-3)
    g = vx.from_workload(w, precision=precision, kernel=vx.KERNEL_FUSED)
    g.write_state(**st)
    g.autotune(iters=1)
    if precision == 32:
        st = g.read_state()          # the FP32-rounded input both sides start from
    g.step(1)
    out = g.read_state()
    rng = np.random.Generator(np.random.PCG64(98))
    picks = [0, n - 1, n * n - 1, ncell - 1, n * n * (n // 2) + n * 5 + 7]
    picks += rng.integers(0, ncell, 43).tolist()
    for c in picks:
        ref = _neighbourhood_oracle(w, st, int(c), n, n, n, g.dt)
        for k in ("u", "v", "w", "q"):
            scale = max(np.abs(ref[k]).max(), np.abs(st[k][c]).max(), 1e-30)
            err = np.abs(out[k][c] - ref[k]).max() / scale
            assert err < tols[k], (c, k, err, out[k][c], ref[k])


@pytest.mark.parametrize("precision", [64, 32])
def test_full_size_random_block_sampled(precision):
    """100^3 random block of the headline benchmark (same grid and
    materials), placed on the floor and moving down at impact speed, in the
    launch configuration bench.py times (fused kernel, autotuned tile): one
    step from a perturbed state, so that about half of the bottom layer
    penetrates the floor (penalty force, ground damping and Coulomb
    friction), then 48 sampled filled voxels (24 of the bottom layer, corners,
    the rest at random) recomputed one by one by the oracle on their
    neighbourhood."""
    tols = FP64_ONE_STEP if precision == 64 else FP32_ONE_STEP
    n = 100
    w = workloads.random_block(n=n, seed=2, impact=True)
    ncell = n ** 3
    announce("full size 100^3 impact p=%d" % precision)
    st = perturbed_state(ncell, 99, 1e-6, 1e-3, 0.5, 1e-3)
    st["v"] = st["v"] + w["velocity"]
    g = vx.from_workload(w, precision=precision, kernel=vx.KERNEL_FUSED)
    g.write_state(**st)
    g.autotune(iters=1)
    if precision == 32:
        st = g.read_state()          # the FP32-rounded input both sides start from
    g.step(1)
    out = g.read_state()
    filled = np.flatnonzero(w["grid"].reshape(-1) > 0)
    bottom = filled[filled < n * n]
    rng = np.random.Generator(np.random.PCG64(100))
    picks = [c for c in (0, n - 1, n * n - 1, ncell - 1) if w["grid"].reshape(-1)[c] > 0]
    picks += rng.choice(bottom, 24, replace=False).tolist()
    picks += rng.choice(filled, 48 - len(picks), replace=False).tolist()
    in_contact = 0
    for c in picks:
        x, y, z = c % n, (c // n) % n, c // (n * n)
        in_contact += int(z == 0 and st["u"][c][2] < 0.0)
        ref = _neighbourhood_oracle(w, st, int(c), n, n, n, g.dt)
        for k in ("u", "v", "w", "q"):
            scale = max(np.abs(ref[k]).max(), np.abs(st[k][c]).max(), 1e-30)
            err = np.abs(out[k][c] - ref[k]).max() / scale
            assert err < tols[k], (c, k, err, out[k][c], ref[k])
    assert in_contact >= 5, in_contact


_CROP = {}


def _blob_crop():
    """The 256^3 lattice's recipe at 48^3 (several tiles of every fused
    shape along x and y) so that the oracle runs all 1000 steps (4
    materials on Voronoi blobs, the 5 Hz thermal actuation from phase 0,
    self-collision on), and the oracle's state after them (computed once
    for both precisions)."""
    if not _CROP:
        w = workloads.blob_lattice(n=48, seed=3)
        o = build_oracle(w)
        assert o.step(1000) == 0
        _CROP["w"], _CROP["ref"] = w, o.read_state()
    return _CROP["w"], _CROP["ref"]


@pytest.mark.parametrize("precision", [64, 32])
def test_blob_lattice_crop_1000_steps(precision):
    """1000 steps of the cropped blob lattice through the fused kernel with
    an autotuned tile: FP64 within 1e-10 of the oracle, FP32 largest
    displacement within 1e-4."""
    w, ref = _blob_crop()
    announce("blob lattice 48^3 x 1000 p=%d" % precision)
    g = build_gpu(w, precision=precision, kernel=vx.KERNEL_FUSED)
    g.autotune(iters=1)
    g.step(1000)
    got = g.read_state()
    f = filled_of(w)
    e = compare(got, ref, f)
    if precision == 64:
        assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12, e
    else:
        ug = np.linalg.norm(got["u"][f], axis=1).max()
        uo = np.linalg.norm(ref["u"][f], axis=1).max()
        assert abs(ug / uo - 1.0) < FP32_MAXDISP_TOL and e["u"] < 1e-3, (ug, uo, e)


def test_appendix_program():
    """The paper's appendix example through the C ABI: a 5x10x5 workspace of
    1 mm voxels of one 10 MPa material (Poisson ratio 0.3), the -y face fixed
    and 1 kN downward on the +y face by the region calls, ground damping
    0.013, 400 steps.  The load is far beyond the beam's strength, so the
    motion turns chaotic after about 100 steps (in the oracle a 1e-18 m
    perturbation stays at 1e-15 of the displacement for 80 steps and reaches
    2e-7 by step 150).  FP64 equals the oracle, whose regions come from its
    own selection code, within 1e-10 over the first 80 steps; all 400 steps
    then run without error, with the fixed layer held."""
    from oracle import regions
    g = np.ones((5, 10, 5), np.uint8)
    mats = [workloads.EMPTY, workloads._mat(1e7, nu=0.3)]
    params = workloads._base_params(zeta_slow=0.013)
    announce("appendix program")
    s = vx.Sim(g, mats, precision=64, **params)
    s.fixed_region((0, 0, 0), (1.0, 0.01, 1.0))
    s.forced_region((0, 0.99, 0), (1.0, 0.01, 1.0), (0, 0, -1000.0))
    o = oracle.Sim(g, mats, **params)
    o.set_fixed(regions.region_mask(g, (0, 0, 0), (1.0, 0.01, 1.0)))
    o.set_forces(regions.forced_region_forces(g, (0, 0.99, 0), (1.0, 0.01, 1.0), (0, 0, -1000.0)))
    s.step(80)
    assert o.step(80) == 0
    e = compare(s.read_state(), o.read_state(), filled_of({"grid": g}))
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12, e
    s.step(320)                      # raises on VX_EUNSTABLE
    st = s.read_state()
    assert all(np.isfinite(st[k]).all() for k in st)
    _, y, _ = workloads.cell_coords(g.shape)
    assert not st["u"][y == 0].any() and np.abs(st["u"][y == 9]).max() > 1e-3
