"""Seeded synthetic inputs for the voxel-lattice step.

This module builds inputs only: material grids, palettes, parameter sets,
fixed masks, external forces and initial velocities.  It holds none of the
method's arithmetic, and both the GPU library's tests and the oracle's tests
draw their inputs from it.  Every random choice goes through
``numpy.random.Generator(PCG64(seed))``.

A workload is a dict:
  grid      uint8 (nz, ny, nx), material index per cell, 0 = empty
  materials list of dicts {E, nu, rho, cte, mu_s, mu_d}; index 0 is empty
  params    dict of simulation parameters (voxel_size, gravity, zeta_*, ...)
  fixed     uint8 per cell or None
  forces    float64 (ncell, 3) or None
  velocity  float64 (ncell, 3) or None
  amp/phase float64 per cell or None (per-voxel actuation signal)
  steps     number of steps the scenario runs
"""
import numpy as np

EMPTY = {"E": 1.0, "nu": 0.0, "rho": 1.0, "cte": 0.0, "mu_s": 0.0, "mu_d": 0.0}


def _mat(E, nu=0.35, rho=1000.0, cte=0.0, mu_s=1.0, mu_d=0.5):
    return {"E": float(E), "nu": float(nu), "rho": float(rho), "cte": float(cte),
            "mu_s": float(mu_s), "mu_d": float(mu_d)}


def _base_params(**kw):
    p = {"voxel_size": 1e-3, "gravity": 0.0, "zeta_bond": 0.0, "zeta_slow": 0.0, "zeta_col": 0.0,
         "temp_amp": 0.0, "temp_freq": 0.0, "temp_phase": 0.0, "dt_scale": 1.0,
         "origin": (0.0, 0.0, 0.0), "floor_on": 0, "self_collision_on": 0, "contact_cap": 32}
    p.update(kw)
    return p


def _workload(grid, materials, params, steps, fixed=None, forces=None, velocity=None,
              amp=None, phase=None, name=""):
    return {"name": name, "grid": np.ascontiguousarray(grid, dtype=np.uint8), "materials": materials,
            "params": params, "steps": int(steps), "fixed": fixed, "forces": forces,
            "velocity": velocity, "amp": amp, "phase": phase}


def cell_coords(shape):
    """(x, y, z) integer index arrays of a (nz, ny, nx) grid, flattened."""
    nz, ny, nx = shape
    c = np.arange(nx * ny * nz)
    return c % nx, (c // nx) % ny, c // (nx * ny)


def cantilever(nx=20, ny=4, nz=4, steps=10000):
    """Cantilever of nx*ny*nz 1 mm voxels, E = 1 MPa, nu = 0.35, rho = 1000,
    x = 0 layer fixed, gravity, light damping."""
    grid = np.ones((nz, ny, nx), np.uint8)
    x, _, _ = cell_coords(grid.shape)
    fixed = (x == 0).astype(np.uint8)
    params = _base_params(gravity=9.81, zeta_bond=0.1, zeta_slow=0.01)
    return _workload(grid, [EMPTY, _mat(1e6)], params, steps, fixed=fixed, name="cantilever_20x4x4")


def thin_beam(nx=20, rho=1.0, zeta_bond=0.01, tip_velocity=1e-3, steps=820000):
    """The paper's dynamic validation beam: nx x 1 x 1 voxels of 1 mm, E =
    1 MPa, nu = 0.35, the x = 0 voxel fixed, no gravity and only the trace
    bond damping zeta_bond; the impulse at the free end is an initial z
    velocity of the tip voxel.  rho = 1 kg/m^3 is the reading under which
    the paper's beam-theory frequencies follow from its formula (the density
    is not stated)."""
    grid = np.ones((1, 1, nx), np.uint8)
    fixed = np.zeros(nx, np.uint8)
    fixed[0] = 1
    v = np.zeros((nx, 3))
    v[nx - 1, 2] = tip_velocity
    params = _base_params(zeta_bond=zeta_bond)
    return _workload(grid, [EMPTY, _mat(1e6, rho=rho)], params, steps, fixed=fixed, velocity=v,
                     name="thin_beam_%dx1x1" % nx)


def random_block(n=100, seed=2, steps=1000, drop_height=5e-3, impact=False):
    """n^3 cells iid {empty 0.1, soft 1 MPa 0.45, stiff 100 MPa 0.45} on a floor
    with friction.  ``impact=False``: the bottom faces at ``drop_height``
    above the floor, at rest.  ``impact=True``: the bottom faces on the
    floor, moving down at the speed of a ``drop_height`` free fall."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = rng.choice(np.array([0, 1, 2], np.uint8), size=(n, n, n), p=[0.1, 0.45, 0.45])
    mats = [EMPTY, _mat(1e6), _mat(1e8)]
    g = 9.81
    l = 1e-3
    # origin = lower corner of cell (0, 0, 0), i.e. the height of the bottom faces
    z0 = 0.0 if impact else drop_height
    params = _base_params(gravity=g, zeta_bond=0.5, zeta_col=0.5, floor_on=1, origin=(0.0, 0.0, z0))
    vel = None
    if impact:
        vel = np.zeros((grid.size, 3))
        vel[:, 2] = -np.sqrt(2.0 * g * drop_height)
    name = "random_block_%d%s" % (n, "_impact" if impact else "")
    return _workload(grid, mats, params, steps, velocity=vel, name=name)


def blob_lattice(n=256, seed=3, steps=500, sites=64, n_mat=4):
    """n^3 lattice, every cell filled, materials assigned by nearest of
    ``sites`` seeded points (Voronoi blobs).  Material k has E log-uniform in
    [0.1, 100] MPa and CTE uniform in [0, 0.01]/K; temperature signal
    20 K sin(2 pi 5 Hz t); self-collision on; no gravity, no floor."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.uniform(0, n, size=(sites, 3))
    lab = rng.integers(0, n_mat, size=sites)
    E = 10.0 ** rng.uniform(5.0, 8.0, size=n_mat)
    cte = rng.uniform(0.0, 0.01, size=n_mat)
    grid = np.empty((n, n, n), np.uint8)
    xs = np.arange(n) + 0.5
    X, Y = np.meshgrid(xs, xs, indexing="xy")  # (ny, nx)
    for z in range(n):
        best = np.full((n, n), np.inf)
        arg = np.zeros((n, n), np.int64)
        for s in range(sites):
            d = (X - pts[s, 0]) ** 2 + (Y - pts[s, 1]) ** 2 + (z + 0.5 - pts[s, 2]) ** 2
            m = d < best
            best[m] = d[m]
            arg[m] = s
        grid[z] = (lab[arg] + 1).astype(np.uint8)
    mats = [EMPTY] + [_mat(E[k], cte=cte[k]) for k in range(n_mat)]
    params = _base_params(zeta_bond=0.5, zeta_col=0.5, temp_amp=20.0, temp_freq=5.0,
                          self_collision_on=1)
    return _workload(grid, mats, params, steps, name="blob_lattice_%d" % n)


def batch_objects(count=4096, seed=4, steps=2000, lo=8, hi=32):
    """``count`` independent objects with bounding boxes iid U{lo..hi} per
    axis, cells iid uniform over {empty, soft, stiff, actuated+, actuated-}
    (actuation: CTE +/-0.01 under a 20 K, 5 Hz signal, i.e. phases 0 and pi),
    each on a floor under gravity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mats = [EMPTY, _mat(1e6), _mat(1e8), _mat(1e6, cte=0.01), _mat(1e6, cte=-0.01)]
    objs = []
    for i in range(count):
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        grid = rng.integers(0, 5, size=(nz, ny, nx)).astype(np.uint8)
        params = _base_params(gravity=9.81, zeta_bond=0.5, zeta_col=0.5, floor_on=1,
                              temp_amp=20.0, temp_freq=5.0)
        objs.append(_workload(grid, mats, params, steps, name="batch_obj_%d" % i))
    return objs


def solid_cube(n, E=1e6, steps=100, **kw):
    """A full n^3 block of one material (performance shape of the paper's
    cubic-block sweep)."""
    grid = np.ones((n, n, n), np.uint8)
    params = _base_params(**kw)
    return _workload(grid, [EMPTY, _mat(E)], params, steps, name="cube_%d" % n)


def random_grid(shape, n_mat, fill, seed):
    """Cells iid: empty with probability 1 - fill, else uniform over 1..n_mat."""
    rng = np.random.Generator(np.random.PCG64(seed))
    filled = rng.uniform(size=shape) < fill
    mat = rng.integers(1, n_mat + 1, size=shape)
    return np.where(filled, mat, 0).astype(np.uint8)


def random_materials(n_mat, seed, cte_max=0.0):
    """Materials with E log-uniform in [0.1, 100] MPa, rho in [500, 2000],
    nu in [0.2, 0.45] and CTE uniform in [-cte_max, cte_max]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = [EMPTY]
    for _ in range(n_mat):
        out.append(_mat(10.0 ** rng.uniform(5, 8), nu=rng.uniform(0.2, 0.45),
                        rho=rng.uniform(500, 2000), cte=rng.uniform(-cte_max, cte_max)))
    return out


def random_state(ncell, seed, u_scale, v_scale, w_scale, rot_scale):
    """Perturbed state: displacements, velocities, angular velocities and small
    rotation vectors drawn iid normal with the given scales."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return {"u": rng.normal(0, u_scale, (ncell, 3)), "v": rng.normal(0, v_scale, (ncell, 3)),
            "w": rng.normal(0, w_scale, (ncell, 3)), "rot": rng.normal(0, rot_scale, (ncell, 3))}


def grad_object(seed, n=4, scenario="free", steps=200, temp_freq=500.0):
    """Small object for gradient checks: an n^3 block in which every voxel
    has its own palette entry (modulus log-uniform in [0.5, 2] MPa, density
    log-uniform in [500, 2000] kg/m^3, CTE 0.01), a per-voxel actuation
    signal (20 K, phase U[0, 2 pi)), and a detached two-voxel anchor of an
    8 MPa, 1000 kg/m^3 material one empty cell beyond +x.  The anchor's bond
    is the fastest (k/m = 8e9 /s^2 against at most 4e9 in the block), so it
    alone sets the timestep: perturbing any block modulus or density leaves
    dt unchanged.

    scenario "free":  no gravity or floor; random initial velocities and
                      spins; two fixed and two forced block voxels; bond
                      and ground damping on.
    scenario "slide": block on the floor under gravity, sliding at 5 cm/s
                      along +x (Coulomb sliding branch), bond and floor
                      damping on.
    scenario "rest":  block on the floor under gravity, at rest (static
                      friction branches).

    Returns a workload plus ``block`` (cell indices of the block voxels,
    ascending), ``E_block`` and ``rho_block`` (their moduli and densities,
    in that order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n + 3, n, n
    grid = np.zeros((nz, ny, nx), np.uint8)
    block = []
    mats = [EMPTY]
    E_block = np.exp(rng.uniform(np.log(0.5e6), np.log(2e6), size=n ** 3))
    rho_block = np.exp(rng.uniform(np.log(500.0), np.log(2000.0), size=n ** 3))
    k = 0
    for z in range(nz):
        for y in range(ny):
            for x in range(n):
                mats.append(_mat(E_block[k], rho=rho_block[k], cte=0.01))
                grid[z, y, x] = len(mats) - 1
                block.append(x + nx * (y + ny * z))
                k += 1
    mats.append(_mat(8e6))
    grid[0, 0, n + 1] = grid[0, 0, n + 2] = len(mats) - 1
    block = np.array(block)
    ncell = grid.size
    amp = np.zeros(ncell)
    amp[block] = 20.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=ncell)
    fixed = forces = velocity = None
    if scenario == "free":
        params = _base_params(zeta_bond=0.3, zeta_slow=0.01, temp_freq=temp_freq)
        velocity = np.zeros((ncell, 3))
        velocity[block] = rng.normal(0.0, 1e-3, size=(block.size, 3))
        fixed = np.zeros(ncell, np.uint8)
        fixed[block[rng.choice(block.size, 2, replace=False)]] = 1
        forces = np.zeros((ncell, 3))
        forces[block[rng.choice(block.size, 2, replace=False)]] = rng.normal(0.0, 1e-4, size=(2, 3))
    elif scenario in ("slide", "rest"):
        params = _base_params(gravity=9.81, zeta_bond=0.3, zeta_col=0.5, floor_on=1, temp_freq=temp_freq)
        if scenario == "slide":
            velocity = np.zeros((ncell, 3))
            velocity[block, 0] = 0.05
    else:
        raise ValueError(scenario)
    w = _workload(grid, mats, params, steps, fixed=fixed, forces=forces, velocity=velocity,
                  amp=amp, phase=phase, name="grad_object_%s_%d" % (scenario, n))
    w["block"] = block
    w["E_block"] = E_block
    w["rho_block"] = rho_block
    return w


def contact_pair(seed, n=3, steps=300, shift=1.4e-3, speed=0.5, temp_freq=500.0):
    """Two n^3 blocks of one lattice that meet: block A at x = 0..n-1, block
    B at x = n+3..2n+2 (rest indices at least 4 apart in Manhattan
    distance, so their voxels may touch), displaced toward each other by
    ``shift`` (m) and moving toward each other at ``speed`` m/s each, so
    that they come into contact after about a third of the run and push
    apart again.  As in grad_object every block voxel has its own palette
    entry (modulus log-uniform in [0.5, 2] MPa, density in [500, 2000]
    kg/m^3, CTE 0.01) and its own actuation phase (20 K), and a detached
    two-voxel 8 MPa anchor beyond B sets the timestep.  Self-collision on,
    no gravity or floor, bond and collision damping on.  Returns a workload
    with ``state`` (the displaced start), ``block``, ``E_block`` and
    ``rho_block``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = 2 * n + 6, n, n
    grid = np.zeros((nz, ny, nx), np.uint8)
    mats = [EMPTY]
    nb = 2 * n ** 3
    E_block = np.exp(rng.uniform(np.log(0.5e6), np.log(2e6), size=nb))
    rho_block = np.exp(rng.uniform(np.log(500.0), np.log(2000.0), size=nb))
    block, side = [], []
    for z in range(nz):
        for y in range(ny):
            for x in list(range(n)) + list(range(n + 3, 2 * n + 3)):
                k = len(block)
                mats.append(_mat(E_block[k], rho=rho_block[k], cte=0.01))
                grid[z, y, x] = len(mats) - 1
                block.append(x + nx * (y + ny * z))
                side.append(1.0 if x < n else -1.0)
    mats.append(_mat(8e6))
    grid[0, 0, 2 * n + 4] = grid[0, 0, 2 * n + 5] = len(mats) - 1
    block = np.array(block)
    order = np.argsort(block)
    block, E_block, rho_block = block[order], E_block[order], rho_block[order]
    side = np.array(side)[order]
    ncell = grid.size
    amp = np.zeros(ncell)
    amp[block] = 20.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=ncell)
    u = np.zeros((ncell, 3)); v = np.zeros((ncell, 3))
    u[block, 0] = side * shift
    v[block, 0] = side * speed
    v[block] += rng.normal(0.0, 0.02 * speed, size=(block.size, 3))
    q = np.zeros((ncell, 4)); q[:, 0] = 1.0
    params = _base_params(zeta_bond=0.3, zeta_col=0.5, self_collision_on=1, contact_cap=64, temp_freq=temp_freq)
    w = _workload(grid, mats, params, steps, amp=amp, phase=phase, name="contact_pair_%d" % n)
    w["state"] = {"u": u, "q": q, "v": v, "w": np.zeros((ncell, 3))}
    w["block"] = block
    w["E_block"] = E_block
    w["rho_block"] = rho_block
    return w


def clapper(freq=20.0, cte=0.02, amp=30.0, gap=5, steps=5000):
    """A clapper for the collision-scheme comparison (section "Speedup of
    self collision schemes"; the paper's geometry is only pictured): a
    two-layer base, fixed at its bottom layer, carrying two 12-voxel arms
    across a gap of ``gap`` cells, each arm a bilayer whose outer layer has
    CTE +cte and inner layer -cte, so that the temperature signal (amp K,
    freq Hz) bends the arms toward each other and apart.  All materials
    1 MPa, self-collision on, no gravity.  cte 0.02 and 30 K are the paper's
    values (60% expansion and contraction); the frequency is not given."""
    nx, ny, nz = gap + 8, 3, 14
    g = np.zeros((nz, ny, nx), np.uint8)
    g[0:2, :, :] = 1
    g[2:, :, 1] = 2
    g[2:, :, 2] = 3
    g[2:, :, nx - 2] = 2
    g[2:, :, nx - 3] = 3
    mats = [EMPTY, _mat(1e6), _mat(1e6, cte=cte), _mat(1e6, cte=-cte)]
    params = _base_params(zeta_bond=0.5, zeta_col=0.5, self_collision_on=1, temp_amp=amp, temp_freq=freq)
    _, _, z = cell_coords(g.shape)
    fixed = ((z == 0) & (g.reshape(-1) > 0)).astype(np.uint8)
    return _workload(g, mats, params, steps, fixed=fixed, name="clapper")


def walker(nx=8, ny=2, nz=2, seed=6, freq=100.0, steps=6000):
    """A soft bar (E = 1 MPa, rho = 1000, CTE 0.01) lying on the floor under
    gravity with friction (mu_s 1, mu_d 0.5), every voxel actuated at 20 K
    and freq Hz with its own phase, U[0, 2 pi) from the seed: the object of
    the gradient-driven design loop (phases tuned for travel along +x).
    Returns a workload plus ``E`` and ``rho`` per cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = np.ones((nz, ny, nx), np.uint8)
    mats = [EMPTY, _mat(1e6, cte=0.01)]
    params = _base_params(gravity=9.81, zeta_bond=0.5, zeta_col=0.5, floor_on=1, temp_freq=freq)
    n = grid.size
    w = _workload(grid, mats, params, steps, amp=np.full(n, 20.0), phase=rng.uniform(0.0, 2 * np.pi, n),
                  name="walker_%dx%dx%d" % (nx, ny, nz))
    w["E"] = np.full(n, 1e6)
    w["rho"] = np.full(n, 1000.0)
    return w


def design_lattice(count=64, size=20, gap=1, seed=5, steps=5000):
    """Many full size^3 design blocks in one lattice, on a sqrt(count) x
    sqrt(count) layout in x-y separated by ``gap`` empty cells (so no bonds
    join them), on the floor under gravity with friction.  Every voxel has
    its own modulus E_v = 1 MPa * 100^sigmoid(s_v) with logits s_v ~ N(0, 1)
    and its own actuation phase U[0, 2 pi) (CTE 0.01, 20 K, 5 Hz).  The
    palette's one material is 100 MPa, the top of the modulus range, so the
    timestep is the one of the stiffest design and does not depend on the
    parameters.  Returns a workload plus ``E`` (per cell) and ``logits``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side = int(round(count ** 0.5))
    assert side * side == count
    pitch = size + gap
    nx = ny = side * pitch - gap
    nz = size
    grid = np.zeros((nz, ny, nx), np.uint8)
    for i in range(side):
        for j in range(side):
            grid[:, j * pitch:j * pitch + size, i * pitch:i * pitch + size] = 1
    mats = [EMPTY, _mat(1e8, cte=0.01)]
    params = _base_params(gravity=9.81, zeta_bond=0.5, zeta_col=0.5, floor_on=1, temp_amp=20.0,
                          temp_freq=5.0)
    ncell = grid.size
    logits = rng.normal(0.0, 1.0, size=ncell)
    E = 1e6 * 100.0 ** (1.0 / (1.0 + np.exp(-logits)))
    E[grid.reshape(-1) == 0] = 0.0
    amp = np.where(grid.reshape(-1) > 0, 20.0, 0.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=ncell)
    w = _workload(grid, mats, params, steps, amp=amp, phase=phase,
                  name="design_lattice_%dx%d" % (count, size))
    w["E"] = E
    w["logits"] = logits
    return w


def colliding_bodies(pairs=(2, 4, 3), seed=7, speed=1.5, steps=1000, lo=3, hi=5, gap=3, slot_yz=9,
                     n_mat=2, spin=50.0, lateral=0.1):
    """Free bodies in approaching pairs: pair slots on a px x py x pz grid,
    each pair two boxes with sides drawn uniformly from lo..hi cells, facing
    each other along x across ``gap`` empty cells and moving towards each
    other at +-speed m/s (plus a seeded lateral velocity of up to
    lateral x speed and a spin of up to ``spin`` rad/s per body).  Cells
    are iid over n_mat materials (E 1 and 5 MPa).  Every two voxels of
    different bodies are more than 3 cells apart in lattice Manhattan
    distance.  No gravity, no floor, self-collision on.

    Returns the workload and a list of bodies (x0, y0, z0, sx, sy, sz) in
    lattice cells."""
    rng = np.random.Generator(np.random.PCG64(seed))
    px, py, pz = pairs
    slot_x = 2 * hi + gap + 4          # pair plus a margin of 4 cells
    nx, ny, nz = px * slot_x, py * slot_yz, pz * slot_yz
    grid = np.zeros((nz, ny, nx), np.uint8)
    vel = np.zeros((grid.size, 3))
    w_init = np.zeros((grid.size, 3))
    bodies = []
    E = [1e6, 5e6][:n_mat]
    for k in range(pz):
        for j in range(py):
            for i in range(px):
                xa = i * slot_x + 2
                sa = rng.integers(lo, hi + 1, size=3)
                sb = rng.integers(lo, hi + 1, size=3)
                # body a ends at x = xa + hi - 1, body b starts gap cells later
                xa0 = xa + hi - sa[0]
                xb0 = xa + hi + gap
                for (x0, s, sign) in ((xa0, sa, 1.0), (xb0, sb, -1.0)):
                    y0 = j * slot_yz + int(rng.integers(0, slot_yz - 4 - s[1] + 1))
                    z0 = k * slot_yz + int(rng.integers(0, slot_yz - 4 - s[2] + 1))
                    blk = rng.integers(1, n_mat + 1, size=(s[2], s[1], s[0])).astype(np.uint8)
                    grid[z0:z0 + s[2], y0:y0 + s[1], x0:x0 + s[0]] = blk
                    v = np.array([sign * speed, 0.0, 0.0]) + rng.uniform(-lateral, lateral, 3) * speed
                    om = rng.uniform(-spin, spin, 3)
                    cells = (np.arange(z0, z0 + s[2])[:, None, None] * ny + np.arange(y0, y0 + s[1])[None, :, None]) * nx \
                        + np.arange(x0, x0 + s[0])[None, None, :]
                    cells = cells.reshape(-1)
                    # rigid-body velocity field about the body's centre
                    cx, cy, cz = x0 + (s[0] - 1) / 2, y0 + (s[1] - 1) / 2, z0 + (s[2] - 1) / 2
                    xs, ys, zs = cell_coords(grid.shape)
                    r = np.stack([xs[cells] - cx, ys[cells] - cy, zs[cells] - cz], 1) * 1e-3
                    vel[cells] = v + np.cross(om, r)
                    w_init[cells] = om
                    bodies.append((int(x0), int(y0), int(z0), int(s[0]), int(s[1]), int(s[2])))
    mats = [EMPTY] + [_mat(e) for e in E]
    params = _base_params(zeta_bond=0.5, zeta_col=0.5, self_collision_on=1, contact_cap=64)
    w = _workload(grid, mats, params, steps, name="colliding_bodies_%dx%dx%d" % pairs)
    q = np.zeros((grid.size, 4))
    q[:, 0] = 1.0
    w["state"] = {"u": np.zeros((grid.size, 3)), "q": q, "v": vel, "w": w_init}
    return w, bodies
