"""Helpers shared by the GPU parity tests: run one seeded workload through the
GPU library and through the oracle, and compare states.

Norm (reading of "relative" in the parity gates): the largest absolute
difference of a quantity divided by the largest magnitude the oracle's
displacement (or that quantity) reaches, so that voxels at rest do not
divide by zero.
"""
import numpy as np

import oracle
import paper_1212_2845_amd as vx


def build_oracle(w):
    o = oracle.Sim(w["grid"], w["materials"], **w["params"])
    if w.get("fixed") is not None:
        o.set_fixed(w["fixed"])
    if w.get("forces") is not None:
        o.set_forces(w["forces"])
    if w.get("amp") is not None or w.get("phase") is not None:
        o.set_actuation(w.get("amp"), w.get("phase"))
    if w.get("velocity") is not None:
        o.set_velocity(w["velocity"])
    if w.get("state") is not None:
        o.write_state(**w["state"])
    return o


def build_gpu(w, precision=64, kernel=vx.KERNEL_FUSED):
    s = vx.from_workload(w, precision=precision, kernel=kernel)
    if w.get("state") is not None:
        s.write_state(**w["state"])
    return s


def rel_err(a, b, scale=None):
    """max |a - b| / scale (scale defaults to max |b|)."""
    a = np.asarray(a); b = np.asarray(b)
    s = np.abs(b).max() if scale is None else scale
    if s == 0:
        return float(np.abs(a - b).max())
    return float(np.abs(a - b).max() / s)


def compare(gpu_state, ora_state, filled, voxel_size=1e-3):
    """Per-quantity relative errors over filled cells.  Displacement and
    velocity use the oracle's largest magnitude of that quantity as scale;
    angular velocity uses the larger of its own largest magnitude and
    max|v| / l (the spin a velocity difference of max|v| across one voxel
    implies), so that a motion without rotation does not divide by rounding
    noise; the quaternion is compared in absolute terms, up to sign."""
    out = {}
    for k in ("u", "v"):
        out[k] = rel_err(gpu_state[k][filled], ora_state[k][filled])
    vmax = np.abs(ora_state["v"][filled]).max() if filled.any() else 0.0
    wscale = max(np.abs(ora_state["w"][filled]).max() if filled.any() else 0.0, vmax / voxel_size)
    out["w"] = rel_err(gpu_state["w"][filled], ora_state["w"][filled], wscale if wscale > 0 else None)
    qg = gpu_state["q"][filled]; qo = ora_state["q"][filled]
    sign = np.where((qg * qo).sum(1, keepdims=True) < 0, -1.0, 1.0)
    out["q"] = float(np.abs(qg * sign - qo).max()) if filled.any() else 0.0
    return out


def perturbed_state(ncell, seed, u_scale, v_scale, w_scale, rot_scale):
    import workloads
    st = workloads.random_state(ncell, seed, u_scale, v_scale, w_scale, rot_scale)
    r = st["rot"]
    a = np.linalg.norm(r, axis=1, keepdims=True)
    q = np.concatenate([np.cos(a / 2), np.sin(a / 2) * r / np.where(a > 0, a, 1)], axis=1)
    return {"u": st["u"], "q": q, "v": st["v"], "w": st["w"]}
