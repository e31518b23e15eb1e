"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every function declared in include/voxsim.h,
validates its inputs, and its host packing (timestep, surface set, region
selection) agrees with the oracle's setup.  No call here launches a kernel.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "voxsim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vx_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = vx.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(vx.EXPORTED) == names


def test_library_has_no_oracle_dependency():
    """The GPU library must not link or embed the oracle."""
    data = open(vx.LIB_PATH, "rb").read()
    assert b"vxo_" not in data
    assert b"liboracle" not in data


def _create(grid, mats, precision=64, **params):
    h = C.c_void_p()
    g = np.ascontiguousarray(grid, np.uint8)
    pal = vx.make_palette(mats)
    prm = vx.make_params(**params)
    rc = vx.lib().vx_create(g.ctypes.data_as(C.c_void_p), g.shape[2], g.shape[1], g.shape[0],
                            C.cast(pal, C.c_void_p), len(mats), C.cast(C.pointer(prm), C.c_void_p),
                            precision, None, C.byref(h))
    return rc, h


M1 = dict(E=1e6, nu=0.35, rho=1000.0, cte=0.0, mu_s=1.0, mu_d=0.5)


@pytest.mark.parametrize("bad", [
    dict(mats=[workloads.EMPTY, dict(M1, E=0.0)]),
    dict(mats=[workloads.EMPTY, dict(M1, E=-1.0)]),
    dict(mats=[workloads.EMPTY, dict(M1, rho=0.0)]),
    dict(mats=[workloads.EMPTY, dict(M1, nu=0.5)]),
    dict(mats=[workloads.EMPTY, dict(M1, nu=-1.0)]),
    dict(precision=16),
    dict(voxel_size=0.0),
    dict(voxel_size=-1e-3),
    dict(dt_scale=1.5),
    dict(zeta_bond=-0.1),
    dict(grid_value=2),
])
def test_create_rejects_bad_input(bad):
    g = np.ones((2, 2, 2), np.uint8)
    if "grid_value" in bad:
        g[1, 1, 1] = bad["grid_value"]
    mats = bad.get("mats", [workloads.EMPTY, M1])
    params = {k: v for k, v in bad.items() if k in ("voxel_size", "dt_scale", "zeta_bond")}
    rc, h = _create(g, mats, precision=bad.get("precision", 64), **params)
    assert rc == vx.VX_EINVAL
    assert not h.value


def test_null_and_zero_sizes_rejected():
    h = C.c_void_p()
    pal = vx.make_palette([workloads.EMPTY, M1])
    prm = vx.make_params()
    g = np.ones(8, np.uint8)
    L = vx.lib()
    for dims in [(0, 2, 2), (2, 0, 2), (2, 2, -1)]:
        rc = L.vx_create(g.ctypes.data_as(C.c_void_p), *dims, C.cast(pal, C.c_void_p), 2,
                         C.cast(C.pointer(prm), C.c_void_p), 64, None, C.byref(h))
        assert rc == vx.VX_EINVAL
    assert L.vx_create(None, 2, 2, 2, C.cast(pal, C.c_void_p), 2, C.cast(C.pointer(prm), C.c_void_p), 64,
                       None, C.byref(h)) == vx.VX_EINVAL
    assert L.vx_step(None, 1) == vx.VX_EINVAL


def test_step_before_bind_is_state_error():
    s = vx.Sim(np.ones((2, 2, 2), np.uint8), [workloads.EMPTY, M1])
    rc = vx.lib().vx_step(s.h, 1)
    assert rc == vx.VX_ESTATE
    assert "bind" in vx.lib().vx_last_error(s.h).decode()


def test_bind_rejects_small_or_misaligned_workspace():
    s = vx.Sim(np.ones((2, 2, 2), np.uint8), [workloads.EMPTY, M1])
    need = s.workspace_bytes()
    assert need > 0
    L = vx.lib()
    assert L.vx_bind_workspace(s.h, C.c_void_p(4096), need - 1) == vx.VX_EINVAL
    assert L.vx_bind_workspace(s.h, C.c_void_p(4096 + 8), need) == vx.VX_EINVAL


@pytest.mark.parametrize("wl", [workloads.cantilever(), workloads.random_block(n=12, seed=5)])
def test_timestep_matches_oracle(wl):
    s = vx.from_workload(wl)
    o = oracle.Sim(wl["grid"], wl["materials"], **wl["params"])
    assert abs(s.dt / o.dt - 1.0) < 1e-15


def test_timestep_heterogeneous_matches_oracle():
    mats = workloads.random_materials(5, seed=7)
    g = workloads.random_grid((6, 7, 8), 5, 0.8, seed=8)
    s = vx.Sim(g, mats)
    o = oracle.Sim(g, mats)
    assert abs(s.dt / o.dt - 1.0) < 1e-15


def test_surface_set_matches_oracle():
    g = workloads.random_grid((9, 8, 7), 2, 0.7, seed=9)
    mats = workloads.random_materials(2, seed=10)
    s = vx.Sim(g, mats)
    o = oracle.Sim(g, mats)
    assert np.array_equal(s.read_flags()["surface"], o.read_flags()["surface"])


def test_initial_state_is_rest():
    g = workloads.random_grid((3, 4, 5), 2, 0.6, seed=3)
    s = vx.Sim(g, workloads.random_materials(2, seed=4))
    st = s.read_state()
    assert np.all(st["u"] == 0) and np.all(st["v"] == 0) and np.all(st["w"] == 0)
    assert np.all(st["q"][:, 0] == 1) and np.all(st["q"][:, 1:] == 0)


def test_write_then_read_state_before_bind_roundtrip():
    g = np.ones((2, 3, 4), np.uint8)
    s = vx.Sim(g, [workloads.EMPTY, M1])
    rng = np.random.default_rng(0)
    u = rng.normal(size=(24, 3)); v = rng.normal(size=(24, 3)); w = rng.normal(size=(24, 3))
    q = rng.normal(size=(24, 4))
    s.write_state(u=u, q=q, v=v, w=w)
    st = s.read_state()
    assert np.allclose(st["u"], u, rtol=1e-15) and np.allclose(st["q"], q, rtol=1e-15)
    assert np.allclose(st["v"], v, rtol=1e-14) and np.allclose(st["w"], w, rtol=1e-14)


def test_fixed_region_selects_one_layer_appendix_program():
    """The appendix program fixes loc (0,0,0) size (1,0.01,1) of a 5x10x5
    workspace: exactly the y = 0 layer is touched."""
    g = np.ones((5, 10, 5), np.uint8)
    s = vx.Sim(g, [workloads.EMPTY, dict(M1, E=1e7, nu=0.3)])
    s.fixed_region((0, 0, 0), (1.0, 0.01, 1.0))
    # fixed voxels get zero momentum; check through a velocity write
    s.set_velocity(np.ones((g.size, 3)))
    v = s.read_state()["v"]
    _, y, _ = workloads.cell_coords(g.shape)
    assert np.all(v[y == 0] == 0.0)
    assert np.all(v[y > 0] == 1.0)


def test_set_forces_rejects_non_finite():
    s = vx.Sim(np.ones((1, 1, 2), np.uint8), [workloads.EMPTY, M1])
    F = np.zeros((2, 3)); F[1, 0] = np.nan
    with pytest.raises(vx.VoxsimError):
        s.set_forces(F)


# --- parameter mode and differentiable rollouts (host-side checks) ----------

def _grad_obj():
    w = workloads.grad_object(seed=3, scenario="free")
    s = vx.from_workload(w, precision=64)
    g = w["grid"].reshape(-1)
    E = np.array([w["materials"][m]["E"] if m else 0.0 for m in g])
    return w, s, E


def test_set_stiffness_validates_moduli():
    w, s, E = _grad_obj()
    s.set_stiffness(E)           # the palette's own moduli
    s.set_stiffness(None)
    for bad in (0.0, -1.0, np.nan, np.inf):
        E2 = E.copy(); E2[w["block"][5]] = bad
        with pytest.raises(vx.VoxsimError) as e:
            s.set_stiffness(E2)
        assert e.value.code == vx.VX_EINVAL
        rho = np.full(E.size, 1000.0); rho[w["block"][5]] = bad
        with pytest.raises(vx.VoxsimError) as e:
            s.set_density(rho)
        assert e.value.code == vx.VX_EINVAL


def test_per_voxel_parameters_rejected_above_the_timestep_bound():
    """The timestep is fixed at create from the fastest bonded pair (here
    the 8 MPa, 1000 kg/m^3 anchor: k/m = 8e9 /s^2); block moduli or
    densities that make a pair faster would be unstable."""
    w, s, E = _grad_obj()
    b = w["block"]
    E2 = E.copy(); E2[b] = 3.9e6
    rho = np.where(w["grid"].reshape(-1) > 0, 1000.0, 0.0)
    s.set_density(rho)
    s.set_stiffness(E2)                 # 3.9e9 /s^2
    E2[b] = 8.2e6
    with pytest.raises(vx.VoxsimError) as e:
        s.set_stiffness(E2)             # 8.2e9 /s^2
    assert e.value.code == vx.VX_EINVAL
    rho[b] = 480.0                      # 3.9e6 / 480e-9 = 8.1e9 /s^2
    with pytest.raises(vx.VoxsimError) as e:
        s.set_density(rho)
    assert e.value.code == vx.VX_EINVAL
    rho[b] = 520.0
    s.set_density(rho)


def test_per_voxel_parameters_with_self_collision():
    # contact takes the per-voxel constants in parameter mode, and gradient
    # rollouts with contact take any checkpoint interval (the binding below
    # fails only for want of the main workspace)
    g = np.ones((3, 3, 3), np.uint8)
    rc, h = _create(g, [workloads.EMPTY, M1], 64, **workloads._base_params(self_collision_on=1))
    assert rc == vx.VX_OK
    E = np.full(27, 1e6)
    assert vx.lib().vx_set_stiffness(h, E.ctypes.data_as(C.c_void_p)) == vx.VX_OK
    rho = np.full(27, M1["rho"])
    assert vx.lib().vx_set_density(h, rho.ctypes.data_as(C.c_void_p)) == vx.VX_OK
    vx.lib().vx_destroy(h)
    s = vx.Sim(g, [workloads.EMPTY, M1], **workloads._base_params(self_collision_on=1))
    L = vx.lib()
    assert L.vx_grad_bind(s.h, C.c_void_p(4096), 1 << 40, 10, 2) == vx.VX_ESTATE
    assert "vx_bind_workspace" in L.vx_last_error(s.h).decode()


def test_grad_calls_need_their_state():
    w, s, E = _grad_obj()
    L = vx.lib()
    # gradient workspace before the main one
    assert L.vx_grad_bind(s.h, None, 0, 10, 2) == vx.VX_ESTATE
    # forward without a gradient workspace, backward without a recorded run
    assert L.vx_grad_forward(s.h, 5) == vx.VX_ESTATE
    assert L.vx_grad_backward(s.h, *([None] * 12)) == vx.VX_ESTATE
    assert L.vx_grad_forward(s.h, 0) == vx.VX_EINVAL


def test_grad_workspace_size_grows_with_checkpoints_and_segment():
    w, s, E = _grad_obj()
    L = vx.lib()
    def nbytes(steps, K):
        n = C.c_uint64()
        assert L.vx_grad_workspace_bytes(s.h, steps, K, C.byref(n)) == vx.VX_OK
        return n.value
    ncell = w["grid"].size
    # per cell: checkpoints and segment slots of 13 FP64 words + 1 flag byte,
    # 6-word bond sums per segment slot, 2 x 13 adjoint words, 6 + 3 words,
    # 4 FP64 accumulators
    per_cell = lambda nck, K: (nck + K) * (13 * 8 + 1) + K * 48 + 26 * 8 + 9 * 8 + 32
    for steps, K in ((100, 10), (100, 7), (5000, 100)):
        nck = -(-steps // K)
        assert nbytes(steps, K) >= per_cell(nck, K) * ncell
        assert nbytes(steps, K) <= per_cell(nck, K) * ncell + 256 * (2 * nck + 3 * K + 20)
    assert nbytes(100, 200) == nbytes(100, 100)
    assert L.vx_grad_workspace_bytes(s.h, 0, 1, C.byref(C.c_uint64())) == vx.VX_EINVAL
    assert L.vx_grad_workspace_bytes(s.h, 10, 0, C.byref(C.c_uint64())) == vx.VX_EINVAL


def test_grad_bind_with_self_collision_needs_only_the_workspace():
    g = np.ones((3, 3, 3), np.uint8)
    rc, h = _create(g, [workloads.EMPTY, M1], 64, **workloads._base_params(self_collision_on=1))
    assert rc == vx.VX_OK
    for K in (1, 2):
        assert vx.lib().vx_grad_bind(h, None, 0, 10, K) == vx.VX_ESTATE
        assert b"vx_bind_workspace" in vx.lib().vx_last_error(h)
    vx.lib().vx_destroy(h)


def test_batch_state_span_limit():
    # the batched kernel addresses one state array (13 words per cell of all
    # objects) through one buffer descriptor: the array must span < 2^32 B
    lim = ((1 << 32) + 13 * 8 - 1) // (13 * 8)   # first FP64 cell count at or over 2^32 B
    mats = [workloads.EMPTY, M1]
    b = vx.Batch([np.zeros((1, 1, lim - 1), np.uint8)], mats, precision=64)
    assert b.n == 1
    with pytest.raises(vx.VoxsimError) as e:
        vx.Batch([np.zeros((1, 1, lim), np.uint8)], mats, precision=64)
    assert e.value.code == vx.VX_EINVAL


def _tiling_work(nx, ny, tx, ty):
    """Brute force over the lanes of every tile of an nx x ny footprint
    (lane t of a tile at x = t mod tx, y = t // tx; 64 lanes a wavefront):
    (wavefronts holding a cell of the footprint, tiles)."""
    waves = tiles = 0
    lanes = np.arange(tx * ty)
    for y0 in range(0, ny, ty):
        for x0 in range(0, nx, tx):
            inside = (x0 + lanes % tx < nx) & (y0 + lanes // tx < ny)
            waves += sum(bool(inside[a:a + 64].any()) for a in range(0, tx * ty, 64))
            tiles += 1
    return waves, tiles


def test_batch_tile_rules():
    # both rules give tiles the batch kernel takes (TX, TY <= 64, TX TY <=
    # 256, within the footprint); rule 0 is the widest rows; rule 1 equals
    # it up to 64 cells across and otherwise evens the tile widths: the same
    # tiles across x, fewer idle lanes (counted here lane by lane)
    shapes = [(33, 30, 3), (64, 64, 1), (65, 3, 2), (70, 3, 2), (8, 8, 8), (100, 1, 1), (130, 20, 2), (200, 9, 1)]
    grids = [np.ones((nz, ny, nx), np.uint8) for nx, ny, nz in shapes]
    b = vx.Batch(grids, [workloads.EMPTY, M1], precision=32)
    tiles = {}
    for rule in (0, 1):
        if rule:
            b.set_tile_rule(rule)
        for i, (nx, ny, nz) in enumerate(shapes):
            r, tx, ty = b.tile(i)
            assert r == rule
            assert 1 <= tx <= min(nx, 64) and 1 <= ty <= min(ny, 64) and tx * ty <= 256, (rule, i, tx, ty)
            assert ty == min(ny, 256 // tx, 64)
            tiles[rule, i] = (tx, ty)
    for i, (nx, ny, nz) in enumerate(shapes):
        (tx0, ty0), (tx1, ty1) = tiles[0, i], tiles[1, i]
        assert tx0 == min(nx, 64)
        assert -(-nx // tx1) == -(-nx // tx0) and tx1 * (-(-nx // tx1)) - nx < -(-nx // tx1)
        if nx <= 64:
            assert (tx1, ty1) == (tx0, ty0)
        else:
            w0, w1 = _tiling_work(nx, ny, tx0, ty0), _tiling_work(nx, ny, tx1, ty1)
            assert w1[0] <= w0[0] and w1[1] <= w0[1], (shapes[i], w0, w1)
    assert tiles[1, 3] == (35, 3) and _tiling_work(70, 3, 35, 3)[0] < _tiling_work(70, 3, 64, 3)[0]
    b.set_tile_rule(0)
    assert b.tile(3) == (0, 64, 3)
    for bad in (-1, 2):
        with pytest.raises(vx.VoxsimError) as e:
            b.set_tile_rule(bad)
        assert e.value.code == vx.VX_EINVAL
    with pytest.raises(vx.VoxsimError):
        b.tile(len(shapes))


def test_modal_helpers():
    # the beam formula at rho = 1 kg/m^3, L = 20 mm gives the printed
    # beam-theory column of Table 2 (section Validation), to its 4-5 digits
    import json
    from paper_1212_2845_amd import modal
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_modes.json")))
    l = 1e-3
    f = modal.beam_frequencies(1e6, l ** 4 / 12.0, 1.0 * l * l, 0.02, n=6)
    for a, b in zip(f, g["beam_theory_hz"]):
        assert abs(a / b - 1.0) < 5e-4, (f, g["beam_theory_hz"])
    # peak finder on tones between FFT bins: 0.13 s of samples, 7.7 Hz bins
    dt, n = 6.5e-6, 20000
    t = np.arange(n) * dt
    tones = [403.7, 2531.2, 7081.3]
    x = sum(a * np.sin(2 * np.pi * ft * t + p) for ft, a, p in zip(tones, [1.0, 0.1, 0.01], [0.3, 1.0, 2.0]))
    got = modal.peaks(x, dt, 3)
    assert len(got) == 3
    for a, b in zip(got, tones):
        assert abs(a / b - 1.0) < 2e-4, (got, tones)


def test_static_solve_workspace_and_state_errors():
    s = vx.Sim(np.ones((2, 3, 4), np.uint8), [workloads.EMPTY, M1])
    n = C.c_uint64()
    L = vx.lib()
    assert L.vx_static_workspace_bytes(s.h, C.byref(n)) == vx.VX_OK
    ncell = 24
    # moduli (2 x 8 B), clamp mask (1 B), load, x, r, z, p, q, diagonal (7 x 48 B) per cell
    assert n.value >= ncell * (16 + 1 + 7 * 48)
    F = np.zeros((ncell, 3))
    it = C.c_int32(); res = C.c_double()
    rc = L.vx_static_solve(s.h, C.c_void_p(4096), n.value, F.ctypes.data_as(C.c_void_p), 1e-10, 100,
                           None, None, C.byref(it), C.byref(res))
    assert rc == vx.VX_ESTATE
    assert L.vx_static_solve(s.h, C.c_void_p(4096), n.value, F.ctypes.data_as(C.c_void_p), 0.0, 100,
                             None, None, None, None) == vx.VX_EINVAL


def test_self_collision_rejects_axes_beyond_packed_indices():
    """The collision search packs rest indices into 21 bits per axis: a
    lattice more than 2^20 cells long on an axis is refused with
    self-collision on, and accepted without it."""
    g = np.ones((1, 1, (1 << 20) + 1), np.uint8)
    with pytest.raises(vx.VoxsimError):
        vx.Sim(g, [workloads.EMPTY, M1], self_collision_on=1)
    vx.Sim(g, [workloads.EMPTY, M1], self_collision_on=0)


def test_contact_cap_is_bounded():
    """Candidate lists are built in LDS, so contact_cap is at most 1024."""
    g = np.ones((2, 2, 2), np.uint8)
    vx.Sim(g, [workloads.EMPTY, M1], self_collision_on=1, contact_cap=1024)
    with pytest.raises(vx.VoxsimError):
        vx.Sim(g, [workloads.EMPTY, M1], self_collision_on=1, contact_cap=1025)
