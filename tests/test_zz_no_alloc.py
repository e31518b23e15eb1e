"""vx_static_solve_noalloc (the static solve in the library's fixed device
scratch, for callers that cannot allocate) against vx_static_solve with a
caller workspace: two calls in a row on the same device, the second on a
smaller lattice, each bitwise equal to the workspace call on the same
lattice; an oversized lattice is refused."""
import numpy as np
import pytest

import paper_1212_2845_amd as vx
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-13


def beam(nx, ny, nz, load):
    g = np.ones((nz, ny, nx), np.uint8)
    x, _, _ = workloads.cell_coords(g.shape)
    fixed = (x == 0).astype(np.uint8)
    F = np.zeros((g.size, 3))
    end = x == nx - 1
    F[end, 2] = load / end.sum()
    F[end, 1] = 0.3 * load / end.sum()
    return g, [workloads.EMPTY, workloads._mat(1e6, nu=0.35), workloads._mat(1e7, nu=0.3)], fixed, F


def solve_both(nx, ny, nz, load, seed):
    g, mats, fixed, F = beam(nx, ny, nz, load)
    rng = np.random.default_rng(seed)
    g = np.where(rng.random(g.shape) < 0.3, 2, 1).astype(np.uint8)   # two materials, all filled
    s = vx.Sim(g, mats, precision=64, **workloads._base_params())
    s.set_fixed(fixed)
    print("[case] no-alloc static solve %dx%dx%d" % (nx, ny, nz), flush=True)
    a = s.static_solve_noalloc(F, rel_tol=TOL, max_iter=100000)
    b = s.static_solve(F, rel_tol=TOL, max_iter=100000)
    return a, b


def test_noalloc_static_solve_equals_workspace_solve_twice():
    big = solve_both(14, 4, 4, -3e-5, 1)
    small = solve_both(9, 3, 2, -1e-5, 2)
    for a, b in (big, small):
        assert a["iters"] == b["iters"] > 0
        assert a["rel_residual"] == b["rel_residual"] < 1e-9
        assert np.array_equal(a["u"], b["u"])
        assert np.array_equal(a["theta"], b["theta"])
        assert np.abs(a["u"]).max() > 0.0
    # the second, smaller call does not see the first call's larger contents
    assert big[0]["u"].shape != small[0]["u"].shape


def test_noalloc_static_solve_refuses_lattice_beyond_scratch():
    n = 60   # 216,000 cells need about 76 MB of conjugate-gradient vectors
    g = np.ones((n, n, n), np.uint8)
    s = vx.Sim(g, [workloads.EMPTY, workloads._mat(1e6)], precision=64, **workloads._base_params())
    with pytest.raises(vx.VoxsimError) as e:
        s.static_solve_noalloc(np.zeros((g.size, 3)))
    assert e.value.code == vx.VX_EINVAL
    assert "too large" in str(e.value)
