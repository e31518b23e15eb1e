"""Named actuation channels (section Volumetric Actuation: several
independent "temperatures", each driving only some materials) on the GPU
against the FP64 oracle: trajectories of lattices driven by channels of
different frequencies and waveforms, and the per-channel phase and
amplitude gradients of the reverse run against central differences of the
oracle."""
import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import workloads
from gradcheck import loss_weights
from parity import build_gpu, build_oracle, compare, perturbed_state

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
CHANNELS = [{"amp": 12.0, "freq": 260.0, "phase": 0.4, "offset": 2.0, "waveform": "triangle"},
            {"amp": 9.0, "freq": 410.0, "phase": 1.3, "offset": 0.0, "waveform": "sine"},
            {"amp": 5.0, "freq": 150.0, "phase": 2.2, "offset": -1.0, "waveform": "square"}]


def announce(msg):
    print("[case] " + msg, flush=True)


def channel_block(shape=(6, 9, 13), seed=121):
    """Four materials (CTE up to 0.01): material 1 on the triangle channel,
    material 2 on the sine channel, a seeded tenth of the cells overridden
    to the square channel, material 3 on per-voxel signals (its own
    amplitude and phase) and material 4 on the global signal; perturbed
    initial state, bond and ground damping."""
    mats = workloads.random_materials(4, seed=seed, cte_max=0.01)
    g = workloads.random_grid(shape, 4, 0.9, seed + 1)
    w = workloads._workload(g, mats, workloads._base_params(zeta_bond=0.3, zeta_slow=0.01, temp_amp=8.0,
                                                            temp_freq=330.0), 300)
    n = g.size
    w["state"] = perturbed_state(n, seed + 2, 2e-6, 2e-3, 1.0, 2e-3)
    rng = np.random.Generator(np.random.PCG64(seed + 3))
    gr = g.reshape(-1)
    w["amp"] = np.where(gr == 3, rng.uniform(5.0, 15.0, n), 8.0)
    w["phase"] = np.where(gr == 3, rng.uniform(0.0, 2 * np.pi, n), 0.0)
    cell = np.full(n, -1, np.int32)
    cell[rng.random(n) < 0.1] = 2
    return w, [-1, 0, 1, -1, -1], cell


def with_channels(w, mat_channel, cell_channel, channels=CHANNELS, precision=64, kernel=vx.KERNEL_FUSED):
    g = build_gpu(w, precision=precision, kernel=kernel)
    g.set_channels(channels, mat_channel=mat_channel, cell_channel=cell_channel)
    o = build_oracle(w)
    o.set_channels(channels, mat_channel=mat_channel, cell_channel=cell_channel)
    return g, o


@pytest.mark.parametrize("kernel", [vx.KERNEL_FUSED, vx.KERNEL_SPLIT])
def test_three_channels_fp64(kernel):
    w, mc, cc = channel_block()
    announce("three channels fp64 kernel=%d" % kernel)
    g, o = with_channels(w, mc, cc, kernel=kernel)
    g.step(300)
    assert o.step(300) == 0
    e = compare(g.read_state(), o.read_state(), w["grid"].reshape(-1) > 0)
    print(e, flush=True)
    assert max(e["u"], e["v"], e["w"]) < FP64_TOL and e["q"] < 1e-12, e


def test_three_channels_fp32_max_displacement():
    w, mc, cc = channel_block(seed=131)
    announce("three channels fp32")
    g, o = with_channels(w, mc, cc, precision=32)
    g.step(300)
    assert o.step(300) == 0
    f = w["grid"].reshape(-1) > 0
    ug = np.linalg.norm(g.read_state()["u"][f], axis=1).max()
    uo = np.linalg.norm(o.read_state()["u"][f], axis=1).max()
    assert abs(ug / uo - 1.0) < 1e-4, (ug, uo)


def test_channels_change_only_their_voxels_drive():
    """Changing one channel's frequency changes the run; a channel no voxel
    follows does not (bitwise)."""
    w, mc, cc = channel_block(seed=141)
    announce("channel isolation")
    base, _ = with_channels(w, mc, cc)
    base.step(100)
    extra = CHANNELS + [{"amp": 50.0, "freq": 999.0, "phase": 0.0, "offset": 3.0, "waveform": "sine"}]
    same, _ = with_channels(w, mc, cc, channels=extra)
    same.step(100)
    other = [dict(c) for c in CHANNELS]
    other[1]["freq"] = 420.0
    diff, _ = with_channels(w, mc, cc, channels=other)
    diff.step(100)
    a, b, c = base.read_state(), same.read_state(), diff.read_state()
    for k in ("u", "q", "v", "w"):
        assert np.array_equal(a[k], b[k]), k
    assert not np.array_equal(a["u"], c["u"])


def _oracle_loss(w, channels, cell, wu, wv):
    o = build_oracle(w)
    o.set_channels(channels, cell_channel=cell)
    assert o.step(w["steps"]) == 0
    st = o.read_state()
    return float((wu * st["u"]).sum() + (wv * st["v"]).sum())


def test_channel_gradients_match_oracle_differences():
    """A 4^3 free block (fixed and forced voxels, bond and ground damping)
    whose voxels follow two channels, a 500 Hz sine and a 320 Hz triangle,
    by cell: dL/dphase and dL/damp of each channel from the reverse run
    equal central differences (h = 1e-4 of the parameter) of the oracle's
    loss, to 1e-4 of the largest gradient of its kind."""
    w = workloads.grad_object(seed=151, scenario="free")
    wu, wv = loss_weights(w, seed=152)
    chans = [{"amp": 20.0, "freq": 500.0, "phase": 0.7, "offset": 0.0, "waveform": "sine"},
             {"amp": 15.0, "freq": 320.0, "phase": 2.0, "offset": 1.0, "waveform": "triangle"}]
    cell = np.full(w["grid"].size, -1, np.int32)
    b = w["block"]
    cell[b[: b.size // 2]] = 0
    cell[b[b.size // 2:]] = 1
    announce("channel gradients")
    s = vx.from_workload(w, precision=64)
    s.set_channels(chans, cell_channel=cell)
    s.grad_bind(w["steps"], 16)
    s.grad_forward(w["steps"])
    g = s.grad_backward(dL_du=wu, dL_dv=wv)
    gc = s.grad_channels()
    # channel voxels carry no per-voxel signal gradient
    assert not g["phase"][b].any() and not g["amp"][b].any()
    fd = {"phase": np.zeros(2), "amp": np.zeros(2)}
    for k in range(2):
        for key, h in (("phase", 1e-4), ("amp", 1e-4 * chans[k]["amp"])):
            up = [dict(c) for c in chans]; dn = [dict(c) for c in chans]
            up[k][key] += h; dn[k][key] -= h
            fd[key][k] = (_oracle_loss(w, up, cell, wu, wv) - _oracle_loss(w, dn, cell, wu, wv)) / (2 * h)
    print("[grad]", gc, fd, flush=True)
    for key in ("phase", "amp"):
        scale = np.abs(fd[key]).max()
        assert scale > 0
        assert np.abs(gc[key] - fd[key]).max() <= 1e-4 * scale, (key, gc[key], fd[key])
