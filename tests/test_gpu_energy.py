"""Energy and momentum reduction (vx_energy) against the oracle's, on the
same state, and conservation of momentum along a GPU run."""
import numpy as np
import pytest

import workloads
from parity import build_gpu, build_oracle, perturbed_state
from test_gpu_parity import hetero_block

pytestmark = pytest.mark.gpu

KEYS = [("kinetic", "ke"), ("elastic", "elastic"), ("gravity", "gravity"), ("floor", "floor")]


def announce(msg):
    print("[case] " + msg, flush=True)


def floor_block(seed=5):
    """Heterogeneous block resting slightly into the floor, under gravity,
    perturbed and actuated: every energy term is non-zero."""
    w = hetero_block(shape=(6, 5, 4), seed=seed)
    w["params"] = dict(w["params"], gravity=9.81, floor_on=1, zeta_col=0.5)
    st = w["state"]
    st["u"][:, 2] -= 3e-6          # press the block into the floor
    return w


def check(gpu, ora, tol):
    for kg, ko in KEYS:
        a, b = gpu[kg], ora[ko]
        assert abs(a - b) <= tol * max(abs(b), 1e-300), (kg, a, b)
    scaleP = max(np.abs(ora["P"]).max(), 1e-300)
    assert np.abs(np.array(gpu["momentum"]) - ora["P"]).max() <= tol * scaleP
    scaleL = max(np.abs(ora["L"]).max(), 1e-300)
    assert np.abs(np.array(gpu["angular_momentum"]) - ora["L"]).max() <= tol * scaleL


@pytest.mark.parametrize("precision,tol", [(64, 1e-11), (32, 2e-4)])
def test_energy_matches_oracle_on_same_state(precision, tol):
    w = floor_block()
    announce("energy same state p=%d" % precision)
    g = build_gpu(w, precision=precision)
    o = build_oracle(w)
    eg, eo = g.energy(), o.energy()
    print(eg, eo, flush=True)
    assert eo["floor"] > 0 and eo["elastic"] > 0 and eo["ke"] > 0
    check(eg, eo, tol)


def test_energy_matches_oracle_after_steps():
    """After 300 steps on both sides (the trajectories agree to 1e-10)."""
    w = floor_block(seed=9)
    announce("energy after 300 steps")
    g = build_gpu(w, precision=64)
    o = build_oracle(w)
    g.step(300)
    assert o.step(300) == 0
    check(g.energy(), o.energy(), 1e-8)


def test_energy_in_parameter_mode_matches_oracle():
    """Per-voxel moduli through vx_set_stiffness vs the same moduli as
    palette entries."""
    w = workloads.grad_object(seed=13, scenario="rest")
    w["state"] = perturbed_state(w["grid"].size, 14, 2e-6, 2e-3, 1.0, 2e-3)
    announce("energy parameter mode")
    g = build_gpu(w, precision=64)
    gr = w["grid"].reshape(-1)
    g.set_stiffness(np.array([w["materials"][m]["E"] if m else 0.0 for m in gr]))
    o = build_oracle(w)
    g.step(50)
    assert o.step(50) == 0
    check(g.energy(), o.energy(), 1e-8)


def test_momentum_conserved_on_gpu():
    """Free body, bond damping on, no gravity, floor or fixed voxels: the
    total momentum stays constant (pair forces are equal and opposite)."""
    w = hetero_block(shape=(7, 6, 5), seed=17)
    w["params"] = dict(w["params"], zeta_slow=0.0)
    announce("momentum conservation")
    g = build_gpu(w, precision=64)
    P0 = np.array(g.energy()["momentum"])
    g.step(1000)
    P1 = np.array(g.energy()["momentum"])
    assert np.abs(P1 - P0).max() <= 1e-12 * np.abs(P0).max()


def test_energy_record_equals_host_sums():
    """The device record (vx_energy_enqueue alternated with
    vx_step_enqueue, one wait at the end) equals vx_energy taken with a
    host wait after every 3 steps on an identical run, to FP64 rounding of
    the different summation order."""
    import torch
    w = floor_block(seed=21)
    announce("energy record vs host sums")
    g = build_gpu(w, precision=64)
    h = build_gpu(w, precision=64)
    rec = g.energy_record(60, every=3).cpu().numpy()
    assert rec.shape == (21, 10)
    for k in range(rec.shape[0]):
        if k:
            h.step(3)
        e = h.energy()
        want = np.array([e["kinetic"], e["elastic"], e["gravity"], e["floor"]] + list(e["momentum"]) +
                        list(e["angular_momentum"]))
        scale = np.maximum(np.abs(want), 1e-300)
        scale[4:7] = max(np.abs(want[4:7]).max(), 1e-300)
        scale[7:10] = max(np.abs(want[7:10]).max(), 1e-300)
        assert (np.abs(rec[k] - want) <= 1e-12 * scale).all(), (k, rec[k], want)
    torch.cuda.synchronize()


def test_energy_record_of_cantilever_matches_oracle():
    """The energy-per-step record of the 20 x 4 x 4 cantilever under gravity
    (the lattice clamped at x = 0), 200 steps in FP64, against the oracle's
    energies after each step."""
    w = workloads.cantilever(steps=200)
    announce("cantilever energy record")
    g = build_gpu(w, precision=64)
    o = build_oracle(w)
    rec = g.energy_record(200).cpu().numpy()
    for k in range(rec.shape[0]):
        if k:
            assert o.step(1) == 0
        eo = o.energy()
        ref = np.array([eo["ke"], eo["elastic"], eo["gravity"], eo["floor"]])
        assert (np.abs(rec[k, :4] - ref) <= 1e-9 * np.maximum(np.abs(ref), 1e-300) + 1e-30).all(), (k, rec[k], ref)
    assert rec[-1, 0] > 0 and rec[-1, 1] > 0          # the beam moves and bends
    assert rec[-1, 2] < rec[0, 2]                       # and sags
