"""Reverse (adjoint) run of the step on the GPU against central differences
of the FP64 oracle.

Expected values come from tests/gradcheck.py: the oracle run with one
modulus or phase perturbed up and down.  Objects are 4^3 blocks in which
every voxel has its own palette entry (workloads.grad_object), in three
regimes: free flight with fixed and forced voxels and ground damping,
sliding on the floor, and resting on the floor (static friction).  The
GPU runs in parameter mode (per-voxel moduli through vx_set_stiffness) with
checkpoint segments that do not divide the step count.
"""
import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import test_gpu_parity
import workloads
from gradcheck import fd_density, fd_direction, fd_modulus, fd_phase, loss_weights, oracle_loss
from parity import build_oracle, compare

pytestmark = pytest.mark.gpu

SCENARIOS = ["free", "slide", "rest"]


def announce(msg):
    print("[case] " + msg, flush=True)


def palette_field(w, key):
    g = w["grid"].reshape(-1)
    return np.array([w["materials"][m][key] if m else 0.0 for m in g])


def gpu_sim(w, precision=64):
    """Parameter mode: the palette's per-voxel moduli and densities given
    as per-cell arrays."""
    s = vx.from_workload(w, precision=precision)
    s.set_stiffness(palette_field(w, "E"))
    s.set_density(palette_field(w, "rho"))
    return s


def gpu_grad(w, wu, wv, precision=64, K=16):
    s = gpu_sim(w, precision)
    s.grad_bind(w["steps"], K)
    s.grad_forward(w["steps"])
    g = s.grad_backward(dL_du=wu, dL_dv=wv)
    st = s.read_state()
    return g, float((wu * st["u"]).sum() + (wv * st["v"]).sum())


def norm_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_parameter_mode_forward_matches_oracle(scenario):
    """Per-voxel moduli through vx_set_stiffness give the oracle's trajectory
    of the same moduli as palette entries."""
    w = workloads.grad_object(seed=7, scenario=scenario)
    announce("parameter-mode forward %s" % scenario)
    s = gpu_sim(w)
    o = build_oracle(w)
    assert abs(s.dt / o.dt - 1) < 1e-15
    s.step(w["steps"])
    assert o.step(w["steps"]) == 0
    e = compare(s.read_state(), o.read_state(), w["grid"].reshape(-1) > 0)
    assert max(e["u"], e["v"], e["w"]) < 1e-10 and e["q"] < 1e-12, e


def per_voxel_params(w, seed):
    """Per-voxel moduli at most the palette's and densities at least its
    (every bond within the timestep's bound)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = w["grid"].reshape(-1)
    E = palette_field(w, "E") * rng.uniform(0.4, 1.0, g.size)
    rho = palette_field(w, "rho") * rng.uniform(1.0, 2.5, g.size)
    return np.where(g > 0, E, 0.0), np.where(g > 0, rho, 0.0)


@pytest.mark.parametrize("kernel", [vx.KERNEL_FUSED, vx.KERNEL_SPLIT])
def test_per_voxel_moduli_and_densities_match_oracle(kernel):
    """Distinct modulus and density in every voxel (parameter mode of the
    fused and of the split kernels) against the oracle given one palette
    material per voxel with those values, the same timestep, 300 steps on
    the floor with gravity, actuation and a perturbed start: FP64 1e-10."""
    w = test_gpu_parity.hetero_block(shape=(6, 6, 6), seed=91)
    w["params"] = dict(w["params"], gravity=9.81, floor_on=1, zeta_col=0.5)
    E, rho = per_voxel_params(w, 92)
    announce("per-voxel moduli vs oracle kernel=%d" % kernel)
    s = vx.from_workload(w, precision=64, kernel=kernel)
    s.set_stiffness(E)
    s.set_density(rho)
    s.write_state(**w["state"])        # velocities to momenta with the voxels' own masses
    g = w["grid"].reshape(-1)
    cells = np.flatnonzero(g)
    assert len(cells) < 255
    mats = [w["materials"][0]] + [dict(w["materials"][g[c]], E=float(E[c]), rho=float(rho[c])) for c in cells]
    grid2 = np.zeros(g.size, np.uint8)
    grid2[cells] = np.arange(1, len(cells) + 1)
    w2 = dict(w, grid=grid2.reshape(w["grid"].shape), materials=mats)
    own = oracle.Sim(w2["grid"], mats, **dict(w["params"], dt_scale=1.0)).dt
    w2["params"] = dict(w["params"], dt_scale=s.dt / own)
    o = build_oracle(w2)
    assert abs(o.dt / s.dt - 1) < 1e-15
    s.step(300)
    assert o.step(300) == 0
    e = compare(s.read_state(), o.read_state(), g > 0)
    assert max(e["u"], e["v"], e["w"]) < 1e-10 and e["q"] < 1e-12, e


@pytest.mark.parametrize("precision,tol", [(64, 1e-12), (32, 1e-5)])
def test_parameter_mode_fused_matches_split(precision, tol):
    """Parameter mode through the fused kernel (several tiles, two z
    chunks) and through the split kernels: the same device arithmetic, equal
    to rounding; the fused kernel bitwise equal run to run."""
    w = test_gpu_parity.hetero_block(shape=(24, 13, 11), seed=93)
    E, rho = per_voxel_params(w, 94)
    announce("parameter mode fused vs split p=%d" % precision)
    out = []
    for kernel in (vx.KERNEL_FUSED, vx.KERNEL_FUSED, vx.KERNEL_SPLIT):
        s = vx.from_workload(w, precision=precision, kernel=kernel)
        s.set_stiffness(E)
        s.set_density(rho)
        s.write_state(**w["state"])
        if kernel == vx.KERNEL_FUSED:
            s.set_fused_tile(2, 6)          # 16 x 16 tiles: 2 x 1 tiles, chunks of 6 slabs
        s.step(200)
        out.append(s.read_state())
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(out[0][k], out[1][k])
    e = compare(out[2], out[0], w["grid"].reshape(-1) > 0)
    assert max(e["u"], e["v"]) < tol and e["q"] < tol, e


def smooth_fd(f, w, wu, wv, keys):
    """Central differences at h = 1e-4 and 1e-6 for each coordinate.  Where
    the two disagree, a friction or contact event lies inside the
    difference interval (the trajectory map has a kink or jump there) and
    the coordinate has no usable expected value; elsewhere the 1e-6 value
    is the derivative."""
    a = np.array([f(w, wu, wv, k, h=1e-4) for k in keys])
    c = np.array([f(w, wu, wv, k, h=1e-6) for k in keys])
    scale = max(np.abs(c).max(), 1e-300)
    return c, np.abs(a - c) <= 1e-5 * scale, scale


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_gradient_matches_oracle_fd_every_coordinate(scenario):
    """dL/dE, dL/drho and dL/dphase of every block voxel vs central
    differences of the oracle, FP64, on the coordinates where the
    trajectory map is smooth (at least 90% of them); error over the largest
    gradient entry of each."""
    w = workloads.grad_object(seed=11, scenario=scenario)
    wu, wv = loss_weights(w, seed=12)
    announce("fd every coordinate %s" % scenario)
    g, L = gpu_grad(w, wu, wv)
    assert abs(L / oracle_loss(w, wu, wv) - 1) < 1e-10
    b = w["block"]
    idx = np.arange(b.size)
    for name, f, keys, an in (("E", fd_modulus, idx, g["E"][b]), ("rho", fd_density, idx, g["rho"][b]),
                              ("phase", fd_phase, b, g["phase"][b])):
        fd, ok, scale = smooth_fd(f, w, wu, wv, keys)
        err = np.abs(an[ok] - fd[ok]).max() / scale
        print("[grad] %s %s err %.3e on %d of %d coordinates" % (scenario, name, err, ok.sum(), ok.size),
              flush=True)
        assert ok.mean() >= 0.9, (name, ok.sum())
        assert err < 1e-4, (name, err)


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_gradient_matches_oracle_fd_directions(scenario):
    """Directional derivatives along 8 random joint directions in (relative
    modulus, relative density, phase), normalised by |g| |d|, with central
    differences at h = 1e-5 and 1e-7; a direction along which the two
    disagree crosses a friction or contact event inside the interval and
    is skipped (at most 2 of 8)."""
    w = workloads.grad_object(seed=21, scenario=scenario)
    wu, wv = loss_weights(w, seed=22)
    announce("fd directions %s" % scenario)
    g, _ = gpu_grad(w, wu, wv, K=33)
    b = w["block"]
    rng = np.random.Generator(np.random.PCG64(23))
    used = 0
    for i in range(8):
        dE = rng.normal(size=b.size)
        dr = rng.normal(size=b.size)
        dp = np.zeros(w["grid"].size); dp[b] = rng.normal(size=b.size)
        gvec = np.concatenate([g["E"][b] * w["E_block"], g["rho"][b] * w["rho_block"], g["phase"][b]])
        dvec = np.concatenate([dE, dr, dp[b]])
        norm = np.linalg.norm(gvec) * np.linalg.norm(dvec)
        an = float(gvec @ dvec)
        fd = fd_direction(w, wu, wv, dE, dp, drho=dr, h=1e-5)
        fd2 = fd_direction(w, wu, wv, dE, dp, drho=dr, h=1e-7)
        if abs(fd - fd2) > 1e-6 * norm:
            continue
        used += 1
        err = abs(an - fd2) / norm
        assert err < 1e-5, (i, an, fd2, err)
    print("[grad] %s directions used %d of 8" % (scenario, used), flush=True)
    assert used >= 6


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_gradient_matches_fp64_reverse_mode_reference(scenario):
    """Every coordinate of dL/dE, dL/drho, dL/dphase and dL/damp, FP64,
    against reverse mode of the torch reference (oracle/torch_ref.py, itself
    pinned to the C oracle).  Both take the derivative on the branches the
    run takes, so this covers the coordinates where central differences
    straddle a friction event too.  Error over each gradient's largest
    entry."""
    import torch
    from oracle import torch_ref
    w = workloads.grad_object(seed=11, scenario=scenario)
    wu, wv = loss_weights(w, seed=12)
    announce("reverse-mode reference %s" % scenario)
    g, _ = gpu_grad(w, wu, wv)
    lat = torch_ref.Lattice(w)
    E = lat.E0.clone().requires_grad_(True)
    rho = lat.rho0.clone().requires_grad_(True)
    ph = lat.phase0.clone().requires_grad_(True)
    amp = lat.amp0.clone().requires_grad_(True)
    u, q, v, om = torch_ref.rollout(lat, w, w["steps"], E=E, rho=rho, phase=ph, amp=amp)
    c = lat.cells
    L = (torch.from_numpy(wu[c]) * u).sum() + (torch.from_numpy(wv[c]) * v).sum()
    L.backward()
    b = w["block"]
    pos = {cc: k for k, cc in enumerate(c)}
    blk = np.array([pos[cc] for cc in b])
    for name, ref in (("E", E.grad), ("rho", rho.grad), ("phase", ph.grad), ("amp", amp.grad)):
        err = norm_err(g[name][b], ref.numpy()[blk])
        print("[grad] %s vs reference %s err %.3e" % (scenario, name, err), flush=True)
        assert err < 1e-11, (name, err)


def test_gradient_of_initial_state_matches_oracle_fd():
    """dL/d(initial velocity) of a few voxels vs central differences."""
    w = workloads.grad_object(seed=31, scenario="free")
    wu, wv = loss_weights(w, seed=32)
    announce("initial-state gradient")
    g, _ = gpu_grad(w, wu, wv)
    b = w["block"]
    rng = np.random.Generator(np.random.PCG64(33))
    scale = np.abs(g["v0"][b]).max()
    for c in rng.choice(b, 6, replace=False):
        for k in range(3):
            h = 1e-6
            vp = w["velocity"].copy(); vp[c, k] += h
            vm = w["velocity"].copy(); vm[c, k] -= h
            wp = dict(w, velocity=vp); wm = dict(w, velocity=vm)
            fd = (oracle_loss(wp, wu, wv) - oracle_loss(wm, wu, wv)) / (2 * h)
            if w["fixed"][c]:
                continue
            assert abs(g["v0"][c, k] - fd) < 1e-6 * scale, (c, k, g["v0"][c, k], fd)


@pytest.mark.parametrize("precision", [64, 32])
def test_checkpoint_interval_does_not_change_gradients(precision):
    """The reverse run recomputes each segment with the forward kernels, so
    any checkpoint interval gives bitwise the same gradients; K = 1 (the
    tape: the forward run stores every state and bond sum, nothing is
    recomputed) too, with the same loss, i.e. the same final state."""
    w = workloads.grad_object(seed=41, scenario="slide", steps=60)
    wu, wv = loss_weights(w, seed=42)
    announce("checkpoint interval p=%d" % precision)
    ref, loss_ref = gpu_grad(w, wu, wv, precision, K=60)
    for K in (1, 7, 100):
        g, loss = gpu_grad(w, wu, wv, precision, K=K)
        assert loss == loss_ref, K
        for k in ("E", "rho", "phase", "amp", "u0", "v0"):
            assert np.array_equal(g[k], ref[k]), (K, k)


def test_parameter_gradients_without_initial_state():
    """A reverse run asked only for the parameter gradients (no initial-state
    outputs) returns the same modulus, density, phase and amplitude
    gradients, bitwise, as one that also returns the initial-state
    gradients; so does one without the final-velocity adjoint, which then
    skips reading the final momenta back."""
    w = workloads.grad_object(seed=71, scenario="free")
    wu, wv = loss_weights(w, seed=72)
    announce("parameter gradients without the initial state")
    for dv in (wv, None):
        out = []
        for full in (True, False):
            s = gpu_sim(w, 64)
            s.grad_bind(w["steps"], 20)
            s.grad_forward(w["steps"])
            out.append(s.grad_backward(dL_du=wu, dL_dv=dv, initial_state=full))
        assert "v0" in out[0] and "v0" not in out[1]
        for k in ("E", "rho", "phase", "amp"):
            assert np.array_equal(out[0][k], out[1][k]), k


def test_rebinding_a_larger_gradient_workspace():
    """A handle whose gradient workspace was bound for a short rollout and
    then again for a longer one (the host staging taken at the first bind
    is kept) gives, bitwise, the gradients of a fresh handle bound once;
    a second reverse run over the same recorded rollout repeats them."""
    w = workloads.grad_object(seed=73, scenario="free")
    wu, wv = loss_weights(w, seed=74)
    announce("gradient workspace bound twice")
    s = gpu_sim(w, 32)
    s.grad_bind(10, 5)
    s.grad_bind(w["steps"], 20)
    fresh = gpu_sim(w, 32)
    fresh.grad_bind(w["steps"], 20)
    out = []
    for h in (s, fresh):
        h.grad_forward(w["steps"])
        out.append(h.grad_backward(dL_du=wu, dL_dv=wv))
    out.append(s.grad_backward(dL_du=wu, dL_dv=wv))
    for k in ("E", "rho", "phase", "amp", "u0", "v0"):
        assert np.array_equal(out[0][k], out[1][k]), k
        assert np.array_equal(out[0][k], out[2][k]), k


def test_tape_forward_equals_plain_forward():
    """The K = 1 forward run (each step written into the next tape slot) ends
    in the state that plain stepping reaches, bitwise, with the step and
    time counters advanced alike, on a lattice of several fused tiles."""
    w = test_gpu_parity.hetero_block(shape=(24, 13, 11), seed=97)
    E, rho = per_voxel_params(w, 98)
    announce("tape forward")
    out = []
    for tape in (False, True):
        s = vx.from_workload(w, precision=32)
        s.set_stiffness(E)
        s.set_density(rho)
        s.write_state(**w["state"])
        if tape:
            s.grad_bind(37, 1)
            s.grad_forward(37)
        else:
            s.step(37)
        out.append((s.read_state(), s.counters()["steps"], s.time))
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


def test_fp32_gradient_close_to_fp64():
    w = workloads.grad_object(seed=51, scenario="slide")
    wu, wv = loss_weights(w, seed=52)
    announce("fp32 vs fp64 gradient")
    g64, _ = gpu_grad(w, wu, wv, 64)
    g32, _ = gpu_grad(w, wu, wv, 32)
    b = w["block"]
    eE, eP = norm_err(g32["E"][b], g64["E"][b]), norm_err(g32["phase"][b], g64["phase"][b])
    eR = norm_err(g32["rho"][b], g64["rho"][b])
    print("[grad] fp32 vs fp64 E %.3e phase %.3e rho %.3e" % (eE, eP, eR), flush=True)
    assert eE < 1e-4 and eP < 1e-4 and eR < 1e-4, (eE, eP, eR)


def test_rollout_autograd_function():
    """torch.autograd through the library's reverse run."""
    import torch
    w = workloads.grad_object(seed=61, scenario="free")
    wu, wv = loss_weights(w, seed=62)
    announce("autograd rollout")
    s = gpu_sim(w)
    s.grad_bind(w["steps"], 16)
    E0 = s  # keep the Sim alive
    E = torch.tensor(palette_field(w, "E"), dtype=torch.float64, requires_grad=True)
    rho = torch.tensor(palette_field(w, "rho"), dtype=torch.float64, requires_grad=True)
    ph = torch.tensor(w["phase"], dtype=torch.float64, requires_grad=True)
    u, v = vx.rollout(s, E, rho, ph, w["amp"], w["steps"])
    L = (torch.from_numpy(wu) * u).sum() + (torch.from_numpy(wv) * v).sum()
    L.backward()
    ref, _ = gpu_grad(w, wu, wv)
    b = w["block"]
    assert np.allclose(E.grad.numpy()[b], ref["E"][b], rtol=1e-12, atol=0)
    assert np.allclose(rho.grad.numpy()[b], ref["rho"][b], rtol=1e-12, atol=0)
    assert np.allclose(ph.grad.numpy()[b], ref["phase"][b], rtol=1e-12, atol=0)
    del E0


def test_rollout_autograd_on_device_with_amplitude():
    """The autograd rollout with every parameter a CUDA tensor (the
    amplitude, 20 K, in FP32, which holds it exactly): gradients arrive on
    the device in each input's dtype, and the actuation amplitude is
    differentiable like the phase."""
    import torch
    w = workloads.grad_object(seed=61, scenario="free")
    wu, wv = loss_weights(w, seed=62)
    announce("autograd rollout on device")
    s = gpu_sim(w)
    s.grad_bind(w["steps"], 16)
    dev = torch.device("cuda", 0)
    E = torch.tensor(palette_field(w, "E"), dtype=torch.float64, device=dev, requires_grad=True)
    rho = torch.tensor(palette_field(w, "rho"), dtype=torch.float64, device=dev, requires_grad=True)
    ph = torch.tensor(w["phase"], dtype=torch.float64, device=dev, requires_grad=True)
    amp = torch.tensor(w["amp"], dtype=torch.float32, device=dev, requires_grad=True)
    u, v = vx.rollout(s, E, rho, ph, amp, w["steps"])
    L = (torch.from_numpy(wu) * u).sum() + (torch.from_numpy(wv) * v).sum()
    L.backward()
    for t in (E, rho, ph, amp):
        assert t.grad is not None and t.grad.device == t.device and t.grad.dtype == t.dtype
    ref, _ = gpu_grad(w, wu, wv)
    b = w["block"]
    assert np.allclose(E.grad.cpu().numpy()[b], ref["E"][b], rtol=1e-12, atol=0)
    assert np.allclose(rho.grad.cpu().numpy()[b], ref["rho"][b], rtol=1e-12, atol=0)
    assert np.allclose(ph.grad.cpu().numpy()[b], ref["phase"][b], rtol=1e-12, atol=0)
    assert np.abs(ref["amp"][b]).max() > 0
    # the FP32 amplitude's gradient is the FP64 one rounded to FP32
    g32 = amp.grad.cpu().numpy().astype(np.float64)[b]
    assert np.abs(g32 - ref["amp"][b]).max() <= 1e-6 * np.abs(ref["amp"][b]).max()


def test_design_lattice_gradient_full_size():
    """The 64 x 20^3 design lattice (5000 steps, FP32, checkpoint every 100
    steps, the bench's configuration), loss = mean x displacement.  The
    blocks share no bond, so each block's gradients must equal those of the
    same block run alone; the small runs are the regime the oracle
    comparisons above cover.  Forward and reverse evaluate a bond that
    crosses a tile edge in a second inlined copy of the same code, which
    the compiler may contract differently, and the block sits on other tile
    edges in the lattice than alone, so the bar is FP32 rounding (1e-5 of
    each gradient's largest entry).  Central
    differences are no check at this size: with half a million voxels on
    a floor, some voxel always sits at the static-friction threshold, where
    the step zeroes its lateral momentum, so the loss jumps inside any
    difference interval."""
    w = workloads.design_lattice()
    n = w["steps"]
    announce("design lattice full size")
    filled = w["grid"].reshape(-1) > 0
    N = int(filled.sum())
    wu = np.zeros((w["grid"].size, 3)); wu[filled, 0] = 1.0 / N
    s = vx.from_workload(w, precision=32)
    s.set_stiffness(w["E"])
    s.grad_bind(n, 100)
    s.grad_forward(n)
    g = s.grad_backward(dL_du=wu)
    del s
    assert np.isfinite(g["E"]).all() and np.isfinite(g["phase"]).all()
    assert np.abs(g["E"][filled]).max() > 0 and np.abs(g["phase"][filled]).max() > 0
    nz, ny, nx = w["grid"].shape
    size, pitch = 20, 21
    for (i, j) in ((0, 0), (3, 5), (7, 7)):
        sl = (slice(None), slice(j * pitch, j * pitch + size), slice(i * pitch, i * pitch + size))
        cells = np.arange(w["grid"].size).reshape(w["grid"].shape)[sl].reshape(-1)
        wb = workloads._workload(w["grid"][sl], w["materials"], w["params"], n, amp=w["amp"][cells],
                                 phase=w["phase"][cells])
        sb = vx.from_workload(wb, precision=32)
        sb.set_stiffness(w["E"][cells])
        sb.grad_bind(n, 100)
        sb.grad_forward(n)
        gb = sb.grad_backward(dL_du=wu[cells])
        for k in ("E", "rho", "phase", "amp", "u0", "v0"):
            scale = np.abs(g[k][cells]).max()
            err = np.abs(gb[k] - g[k][cells]).max() / scale if scale > 0 else np.abs(gb[k]).max()
            print("[grad] block (%d, %d) %s alone vs in lattice %.3e" % (i, j, k, err), flush=True)
            assert err < 1e-5, (i, j, k, err)


def contact_grad(w, wu, wv, precision=64, K=1, every_step=False):
    s = gpu_sim(w, precision)
    if every_step:
        s.set_collision_mode(all_voxels=0, every_step=1)
    s.write_state(**w["state"])
    s.grad_bind(w["steps"], K)
    s.grad_forward(w["steps"])
    g = s.grad_backward(dL_du=wu, dL_dv=wv)
    st = s.read_state()
    return g, float((wu * st["u"]).sum() + (wv * st["v"]).sum()), s.counters()


def test_gradient_through_contact_matches_oracle_fd():
    """Two blocks of per-voxel moduli, densities and actuation phases pushed
    into each other and apart again (self-collision on, 300 FP64 steps, the
    full tape): the loss equals the oracle's, contact changes it, and dL/dE,
    dL/drho and dL/dphase of every block voxel equal central differences of
    the oracle (which perturbs the voxel's palette entry, i.e. its contact
    stiffness and damping too) on the coordinates where the trajectory map
    is smooth (at least 80% of them), to 1e-4 of the largest entry."""
    w = workloads.contact_pair(seed=61)
    wu, wv = loss_weights(w, seed=62)
    announce("gradient through contact")
    g, L, cnt = contact_grad(w, wu, wv)
    assert abs(L / oracle_loss(w, wu, wv) - 1) < 1e-10
    assert cnt["rebuilds"] >= 2
    w_off = dict(w, params=dict(w["params"], self_collision_on=0))
    assert abs(oracle_loss(w_off, wu, wv) / L - 1) > 1e-3        # the contact matters
    b = w["block"]
    idx = np.arange(b.size)
    for name, f, keys, an in (("E", fd_modulus, idx, g["E"][b]), ("rho", fd_density, idx, g["rho"][b]),
                              ("phase", fd_phase, b, g["phase"][b])):
        fd, ok, scale = smooth_fd(f, w, wu, wv, keys)
        err = np.abs(an[ok] - fd[ok]).max() / scale
        print("[grad] contact %s err %.3e on %d of %d coordinates" % (name, err, ok.sum(), ok.size), flush=True)
        assert ok.mean() >= 0.8, (name, ok.sum())
        assert err < 1e-4, (name, err)


def _with_stiff_anchor(w, E=1e7):
    """Copy of workload w with a bonded pair of voxels of a much stiffer
    material added where the lattice is empty for 4 cells around, so that
    the stable timestep (set by the stiffest bond) does not move when the
    other materials' moduli or densities are perturbed."""
    nz, ny, nx = w["grid"].shape
    grid = w["grid"].copy()
    occ = grid > 0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx - 1):
                zs, ys, xs = slice(max(z - 4, 0), z + 5), slice(max(y - 4, 0), y + 5), slice(max(x - 4, 0), x + 6)
                if not occ[zs, ys, xs].any():
                    grid[z, y, x] = grid[z, y, x + 1] = len(w["materials"])
                    mats = list(w["materials"]) + [workloads._mat(E)]
                    return dict(w, grid=grid, materials=mats)
    raise AssertionError("no room for the anchor")


@pytest.mark.parametrize("rho2", [1000.0, 1300.0])
def test_gradient_through_many_contacts_matches_material_fd(rho2):
    """Eight pairs of free bodies driven into each other (two materials,
    many contacts and several candidate-list rebuilds, FP64, full tape and
    checkpoints every 25 steps; a stiff anchor pair fixes the timestep; the
    materials' densities equal or not): the
    loss equals the oracle's, the two reverse runs agree bitwise, and the
    per-voxel gradients summed over each body material equal central
    differences of the oracle with respect to that material's modulus and
    density (a perturbed palette entry changes every voxel of the material,
    in the bonds and in the contact law)."""
    w, _ = workloads.colliding_bodies(pairs=(2, 2, 2), steps=700)
    # with equal densities (1000) every bond and pair across the materials
    # sits at the kink of the lighter-mass rule, where the central
    # difference and the reverse run both take the mean of the two sides
    w = dict(w, materials=[dict(m) for m in w["materials"]])
    w["materials"][2]["rho"] = rho2
    w = _with_stiff_anchor(w)
    g = w["grid"].reshape(-1)
    filled = g > 0
    rng = np.random.Generator(np.random.PCG64(81))
    wu = np.zeros((g.size, 3)); wv = np.zeros((g.size, 3))
    wu[filled] = rng.normal(0.0, 1.0, size=(filled.sum(), 3))
    wv[filled] = rng.normal(0.0, 1e-3, size=(filled.sum(), 3))
    announce("gradient through many contacts")
    out = []
    for K in (1, 25):
        gr, L, cnt = contact_grad(w, wu, wv, 64, K=K)
        out.append((gr, L, cnt))
    (g1, L1, c1), (g25, L25, c25) = out
    assert c1["rebuilds"] >= 2 and c1["rebuilds"] == c25["rebuilds"]
    assert abs(L1 / oracle_loss(w, wu, wv) - 1) < 1e-10
    w_off = dict(w, params=dict(w["params"], self_collision_on=0))
    assert abs(oracle_loss(w_off, wu, wv) / L1 - 1) > 1e-2        # the bodies do collide
    for k in ("E", "rho", "phase", "amp"):
        assert np.array_equal(g1[k], g25[k]), k

    def fd(key, m, h):
        vals = []
        for sgn in (1.0, -1.0):
            mats = [dict(x) for x in w["materials"]]
            mats[m][key] *= 1.0 + sgn * h
            vals.append(oracle_loss(dict(w, materials=mats), wu, wv))
        return (vals[0] - vals[1]) / (2.0 * h * w["materials"][m][key])

    usable = 0
    for key in ("E", "rho"):
        for m in (1, 2):
            an = g1[key][g == m].sum()
            a, c = fd(key, m, 1e-4), fd(key, m, 1e-5)
            print("[grad] many contacts d/d%s[%d]: analytic %.6e fd %.6e / %.6e" % (key, m, an, a, c), flush=True)
            if abs(a - c) > 1e-4 * abs(a):
                continue           # a contact event inside the difference interval
            usable += 1
            assert abs(an - a) < 1e-4 * abs(a), (key, m, an, a)
    assert usable >= 3, usable


def test_fp32_gradient_through_contact_close_to_fp64():
    """The same two colliding blocks in FP32: the contact branch taken (the
    rebuild count) and the gradients agree with the FP64 run's, relative
    to the largest entry."""
    w = workloads.contact_pair(seed=61)
    wu, wv = loss_weights(w, seed=62)
    announce("fp32 vs fp64 gradient through contact")
    g64, L64, c64 = contact_grad(w, wu, wv, 64)
    g32, L32, c32 = contact_grad(w, wu, wv, 32)
    assert c32["rebuilds"] == c64["rebuilds"]
    assert abs(L32 / L64 - 1) < 1e-4, (L32, L64)
    b = w["block"]
    errs = {k: norm_err(g32[k][b], g64[k][b]) for k in ("E", "rho", "phase")}
    print("[grad] contact fp32 vs fp64 %s" % errs, flush=True)
    assert max(errs.values()) < 1e-4, errs


@pytest.mark.parametrize("K,every_step", [(7, False), (60, False), (7, True)])
def test_checkpointed_gradient_through_contact_equals_tape(K, every_step):
    """With checkpoints every K steps the segment recompute builds candidate
    lists where the forward rebuilt them (by the horizon rule, or every
    step) and at each segment's first step; such lists hold every pair in
    contact, as the forward's did: the recomputed states, and so the
    gradients through contact, are bitwise those of the full tape."""
    w = workloads.contact_pair(seed=61)
    wu, wv = loss_weights(w, seed=62)
    announce("gradient through contact with K = %d, every step %d" % (K, every_step))
    g1, L1, c1 = contact_grad(w, wu, wv, 64, K=1, every_step=every_step)
    gk, Lk, ck = contact_grad(w, wu, wv, 64, K=K, every_step=every_step)
    assert Lk == L1 and ck["rebuilds"] == c1["rebuilds"]
    for k in ("E", "rho", "phase", "amp", "u0", "v0"):
        assert np.array_equal(gk[k], g1[k]), k


def test_tape_forward_with_contact_equals_plain_forward():
    """The K = 1 forward run with self-collision (lists rebuilt by the
    horizon rule, contact forces each step) ends in the state plain
    stepping reaches, bitwise, with the same rebuild count."""
    w = workloads.contact_pair(seed=63)
    announce("tape forward with contact")
    out = []
    for tape in (False, True):
        s = gpu_sim(w, 64)
        s.write_state(**w["state"])
        if tape:
            s.grad_bind(w["steps"], 1)
            s.grad_forward(w["steps"])
        else:
            s.step(w["steps"])
        out.append((s.read_state(), s.counters()["rebuilds"]))
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert out[0][1] == out[1][1] >= 2
