"""Expected gradients for the adjoint tests: central differences of the FP64
oracle.

The loss is linear in the final state, L = sum(wu * u) + sum(wv * v) over
the block voxels, so its gradient with respect to a parameter is the
derivative of the oracle's trajectory map.  Each per-voxel modulus is a
palette entry of its own in the workloads these helpers take
(workloads.grad_object), so perturbing one voxel's modulus or density is
perturbing one palette entry; the actuation phase is the oracle's per-voxel
phase.
"""
import numpy as np

import oracle
from parity import build_oracle


def loss_weights(w, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ncell = w["grid"].size
    wu = np.zeros((ncell, 3)); wv = np.zeros((ncell, 3))
    b = w["block"]
    wu[b] = rng.normal(0.0, 1.0, size=(b.size, 3))
    wv[b] = rng.normal(0.0, 1e-3, size=(b.size, 3))
    return wu, wv


def with_params(w, E_block=None, phase=None, rho_block=None):
    """Copy of workload w with the block moduli, densities and/or phases
    replaced."""
    w2 = dict(w)
    if E_block is not None or rho_block is not None:
        mats = [dict(m) for m in w["materials"]]
        g = w["grid"].reshape(-1)
        for k, c in enumerate(w["block"]):
            if E_block is not None:
                mats[g[c]]["E"] = float(E_block[k])
            if rho_block is not None:
                mats[g[c]]["rho"] = float(rho_block[k])
        w2["materials"] = mats
    if phase is not None:
        w2["phase"] = phase
    return w2


def oracle_loss(w, wu, wv, steps=None):
    o = build_oracle(w)
    rc = o.step(w["steps"] if steps is None else steps)
    assert rc == 0
    st = o.read_state()
    return float((wu * st["u"]).sum() + (wv * st["v"]).sum())


def fd_modulus(w, wu, wv, k, h=1e-4):
    """dL/dE of block voxel k, central difference with relative step h."""
    E = w["E_block"]
    Ep = E.copy(); Ep[k] *= 1.0 + h
    Em = E.copy(); Em[k] *= 1.0 - h
    return (oracle_loss(with_params(w, E_block=Ep), wu, wv) -
            oracle_loss(with_params(w, E_block=Em), wu, wv)) / (2.0 * h * E[k])


def fd_density(w, wu, wv, k, h=1e-4):
    """dL/drho of block voxel k, central difference with relative step h."""
    r = w["rho_block"]
    rp = r.copy(); rp[k] *= 1.0 + h
    rm = r.copy(); rm[k] *= 1.0 - h
    return (oracle_loss(with_params(w, rho_block=rp), wu, wv) -
            oracle_loss(with_params(w, rho_block=rm), wu, wv)) / (2.0 * h * r[k])


def fd_phase(w, wu, wv, c, h=1e-4):
    """dL/dphase of cell c, central difference with step h (radians)."""
    p = w["phase"]
    pp = p.copy(); pp[c] += h
    pm = p.copy(); pm[c] -= h
    return (oracle_loss(with_params(w, phase=pp), wu, wv) -
            oracle_loss(with_params(w, phase=pm), wu, wv)) / (2.0 * h)


def fd_direction(w, wu, wv, dE, dphase, drho=None, h=1e-4):
    """Directional derivative along (relative modulus change dE, phase
    change dphase, relative density change drho)."""
    E = w["E_block"]; p = w["phase"]; r = w["rho_block"]
    dr = np.zeros_like(r) if drho is None else drho
    wp = with_params(w, E_block=E * (1.0 + h * dE), phase=p + h * dphase, rho_block=r * (1.0 + h * dr))
    wm = with_params(w, E_block=E * (1.0 - h * dE), phase=p - h * dphase, rho_block=r * (1.0 - h * dr))
    return (oracle_loss(wp, wu, wv) - oracle_loss(wm, wu, wv)) / (2.0 * h)
