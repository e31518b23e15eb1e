"""Static validation on the GPU (section Validation, Table 1): cantilevers
relaxed to equilibrium, convergence detected from the kinetic energy
reduction, compared with the oracle relaxed for the same number of steps,
with the independent linear direct-stiffness solve and with the paper's
printed deflections."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1212_2845_amd as vx
import workloads
from oracle import ds_solve
from paper_1212_2845_amd import statics

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
L_VOX = 1e-3


def cantilever(shape, load, nu, zeta_slow, zeta_bond):
    nz, ny, nx = shape
    g = np.ones(shape, np.uint8)
    x, _, _ = workloads.cell_coords(shape)
    fixed = (x == 0).astype(np.uint8)
    F = np.zeros((g.size, 3))
    end = x == nx - 1
    F[end, 2] = load / end.sum()
    mats = [workloads.EMPTY, workloads._mat(1e6, nu=nu)]
    params = workloads._base_params(zeta_slow=zeta_slow, zeta_bond=zeta_bond)
    return g, mats, params, fixed, F, end


def relax_both(shape, load, nu, zeta_slow, zeta_bond, rel_tol):
    g, mats, params, fixed, F, end = cantilever(shape, load, nu, zeta_slow, zeta_bond)
    s = vx.Sim(g, mats, precision=64, **params)
    s.set_fixed(fixed)
    s.set_forces(F)
    r = statics.relax(s, rel_tol=rel_tol, chunk=2000, max_steps=400000)
    assert r["converged"], r["history"][-3:]
    o = oracle.Sim(g, mats, **params)
    o.set_fixed(fixed)
    o.set_forces(F)
    assert o.step(r["steps"]) == 0
    return s.read_state()["u"], o.read_state()["u"], g, mats, fixed, F, end, r


def test_thin_beam_table1_on_gpu():
    t = json.load(open(os.path.join(HERE, "golden", "table1_cantilever.json")))
    ug, uo, *_ , r = relax_both((1, 1, 20), -3e-5, 0.35, 2.8e-3, 0.0, 1e-14)
    # the GPU and the oracle took the same steps: FP64 parity
    assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()
    tip_mm = -ug[19, 2] * 1e3
    assert abs(tip_mm - t["thin"]["mass_spring"]) <= 0.0005 + 1e-9


def test_thick_beam_small_load_equals_direct_stiffness_on_gpu():
    ug, uo, g, mats, fixed, F, end, r = relax_both((5, 5, 10), -1e-6, 0.3, 0.01, 0.1, 1e-14)
    # the displacements here are 5e-6 of the voxel size, so rounding at the
    # scale of the voxel weighs 2e5 times more against them than in the
    # 1000-step gates: 1e-9 of the largest displacement
    assert np.abs(ug - uo).max() <= 1e-9 * np.abs(uo).max()
    U, _ = ds_solve.solve(g, mats, L_VOX, fixed, F)
    assert np.abs(ug - U).max() <= 1e-6 * np.abs(U).max()


def test_thick_beam_table1_on_gpu():
    """The 10x5x5 beam at the paper's 0.1 N: the nonlinear relaxation ends
    below the linear solve and within 2% of the printed 0.538 mm (soft pin,
    as for the oracle)."""
    t = json.load(open(os.path.join(HERE, "golden", "table1_cantilever.json")))
    ug, uo, g, mats, fixed, F, end, r = relax_both((5, 5, 10), -0.1, 0.3, 0.01, 0.1, 1e-14)
    assert np.abs(ug - uo).max() <= 1e-10 * np.abs(uo).max()
    U, _ = ds_solve.solve(g, mats, L_VOX, fixed, F)
    tip = -ug[end, 2].mean() * 1e3
    assert tip < -U[end, 2].mean() * 1e3
    assert abs(tip / t["thick"]["mass_spring"] - 1.0) < 0.02


def test_bond_damping_lowers_the_fp32_noise_floor():
    """Section "Effects of local bond damping": with ground damping on, bond
    damping lowers the residual jitter of a relaxed structure.  The C1
    cantilever under gravity in FP32, 100,000 steps: the kinetic-energy
    floor (median of the last 20 checks, over the elastic energy) with
    zeta_bond = 1 lies well below the one with zeta_bond = 0 (measured 8.6x;
    the paper reports about 7 orders of magnitude for its own
    implementation, whose precision is not stated)."""
    floors = {}
    for zb in (0.0, 1.0):
        w = workloads.cantilever()
        w["params"]["zeta_bond"] = zb
        s = vx.from_workload(w, precision=32)
        r = statics.relax(s, rel_tol=0.0, chunk=2000, max_steps=100000)
        h = np.array(r["history"])
        floors[zb] = np.median(h[-20:, 1] / h[-20:, 2])
    print("[case] KE/U floor zeta_bond 0: %.3g, 1: %.3g" % (floors[0.0], floors[1.0]), flush=True)
    assert floors[1.0] * 3.0 < floors[0.0]
