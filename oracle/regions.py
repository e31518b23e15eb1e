"""Region selection of the paper's setup calls (appendix, function
definitions: AddFixedRegion and AddForcedRegion).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

A region is an axis-aligned box given in fractions of the workspace: its
corner `loc` and its extent `size`, each in [0, 1] per axis, where the
workspace spans nx, ny, nz voxels.  The paper says a region acts on the voxels
it touches; touching is read as the voxel's cube and the box sharing a
positive volume, so a box that only meets a voxel along a face, an edge or a
corner does not touch it.  Only filled cells are selected.
"""
import numpy as np


def region_mask(grid, loc, size):
    """uint8 mask (nz*ny*nx, x fastest) of the filled cells whose cube overlaps
    the box [loc, loc + size] (workspace fractions) with positive volume."""
    grid = np.asarray(grid)
    nz, ny, nx = grid.shape
    touched = np.ones(grid.shape, dtype=bool)
    # per axis, in units of voxels: cell k spans [k, k + 1]; the box spans
    # [lo, hi]; they overlap with positive length iff k < hi and k + 1 > lo
    for axis, n, f0, df in ((2, nx, loc[0], size[0]), (1, ny, loc[1], size[1]), (0, nz, loc[2], size[2])):
        lo, hi = f0 * n, (f0 + df) * n
        k = np.arange(n)
        ok = (k < hi) & (k + 1 > lo) & (hi > lo)
        shape = [1, 1, 1]
        shape[axis] = n
        touched &= ok.reshape(shape)
    return (touched & (grid > 0)).reshape(-1).astype(np.uint8)


def forced_region_forces(grid, loc, size, force):
    """Forces (ncell x 3, N) of one forced region: the total `force` split
    equally over the filled cells the region touches, zero elsewhere."""
    m = region_mask(grid, loc, size).astype(bool)
    F = np.zeros((m.size, 3))
    if m.any():
        F[m] = np.asarray(force, dtype=np.float64) / m.sum()
    return F
