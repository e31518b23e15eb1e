"""Linear direct-stiffness solution of a voxel lattice (TEST INFRASTRUCTURE ONLY).

The paper validates its relaxation results against "a linear direct stiffness
method" on the same lattice (section Validation, Table 1).  This module
assembles the 12-DOF beam stiffness of Eq. (7), with the constants of
Eq. (8)-(12), for every face-adjacent voxel pair, rotates each element from the
+x orientation onto its lattice axis, and solves K u = f with numpy.  It is a
second, independent route to the small-load limit of the oracle's stepper.
"""
import numpy as np


def element_stiffness(Ec, Gc, l):
    """Eq. (7): the 12x12 beam stiffness for an element along +x.

    DOF order (X1, Y1, Z1, thx1, thy1, thz1, X2, Y2, Z2, thx2, thy2, thz2).
    """
    A = l * l
    Is = l ** 4 / 12.0
    J = l ** 4 / 6.0
    a1 = Ec * A / l
    a2 = Gc * J / l
    b1 = 12.0 * Ec * Is / l ** 3
    b2 = 6.0 * Ec * Is / l ** 2
    b3 = 2.0 * Ec * Is / l
    K = np.zeros((12, 12))
    # upper triangle exactly as printed (rows 1..12, 0-based here)
    K[0, 0] = a1; K[0, 6] = -a1
    K[1, 1] = b1; K[1, 5] = b2; K[1, 7] = -b1; K[1, 11] = b2
    K[2, 2] = b1; K[2, 4] = -b2; K[2, 8] = -b1; K[2, 10] = -b2
    K[3, 3] = a2; K[3, 9] = -a2
    K[4, 4] = 2 * b3; K[4, 8] = b2; K[4, 10] = b3
    K[5, 5] = 2 * b3; K[5, 7] = -b2; K[5, 11] = b3
    K[6, 6] = a1
    K[7, 7] = b1; K[7, 11] = -b2
    K[8, 8] = b1; K[8, 10] = b2
    K[9, 9] = a2
    K[10, 10] = 2 * b3
    K[11, 11] = 2 * b3
    return np.triu(K) + np.triu(K, 1).T


def _axis_rotation(axis):
    """Matrix taking world vectors into the local frame whose +x is the bond
    axis (a cyclic permutation of the coordinates)."""
    order = [(0, 1, 2), (1, 2, 0), (2, 0, 1)][axis]
    R = np.zeros((3, 3))
    for i, j in enumerate(order):
        R[i, j] = 1.0
    return R


def assemble(grid, materials, l):
    """Global stiffness (6 DOF per filled voxel) of the lattice.

    grid: uint8 (nz, ny, nx); materials: list of dicts with E and nu.
    Returns (K, vox_cells) with vox_cells[k] the dense cell index of DOF block k.
    """
    nz, ny, nx = grid.shape
    flat = grid.reshape(-1)
    cells = np.nonzero(flat)[0]
    index = -np.ones(flat.size, np.int64)
    index[cells] = np.arange(cells.size)
    n = cells.size
    K = np.zeros((6 * n, 6 * n))
    for k, c in enumerate(cells):
        x = c % nx; y = (c // nx) % ny; z = c // (nx * ny)
        for axis, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
            x2, y2, z2 = x + dx, y + dy, z + dz
            if x2 >= nx or y2 >= ny or z2 >= nz:
                continue
            c2 = x2 + nx * (y2 + ny * z2)
            j = index[c2]
            if j < 0:
                continue
            m1 = materials[flat[c]]; m2 = materials[flat[c2]]
            E1, E2 = m1["E"], m2["E"]
            G1 = E1 / (2 * (1 + m1["nu"])); G2 = E2 / (2 * (1 + m2["nu"]))
            Ec = 2 * E1 * E2 / (E1 + E2)           # Eq. (1)
            Gc = 2 * G1 * G2 / (G1 + G2)           # Eq. (2)
            Ke = element_stiffness(Ec, Gc, l)
            R = _axis_rotation(axis)
            T = np.kron(np.eye(4), R)
            Kw = T.T @ Ke @ T
            dofs = np.r_[6 * k:6 * k + 6, 6 * j:6 * j + 6]
            K[np.ix_(dofs, dofs)] += Kw
    return K, cells


def solve(grid, materials, l, fixed_mask, forces):
    """Static displacements under nodal forces with fixed voxels clamped.

    fixed_mask: per cell (flattened), forces: (ncell, 3).  Returns u (ncell, 3)
    and rotations (ncell, 3).
    """
    K, cells = assemble(grid, materials, l)
    n = cells.size
    f = np.zeros(6 * n)
    fm = np.asarray(fixed_mask).reshape(-1)
    F = np.asarray(forces, dtype=np.float64).reshape(-1, 3)
    free = np.ones(6 * n, bool)
    for k, c in enumerate(cells):
        f[6 * k:6 * k + 3] = F[c]
        if fm[c]:
            free[6 * k:6 * k + 6] = False
    u = np.zeros(6 * n)
    u[free] = np.linalg.solve(K[np.ix_(free, free)], f[free])
    ncell = grid.size
    U = np.zeros((ncell, 3)); TH = np.zeros((ncell, 3))
    U[cells] = u.reshape(n, 6)[:, :3]
    TH[cells] = u.reshape(n, 6)[:, 3:]
    return U, TH
