"""Oracle of the voxel-lattice step (Hiller & Lipson, arXiv 1212.2845).

TEST INFRASTRUCTURE ONLY.  A ctypes binding to the plain C FP64 stepper in
``vx_oracle.c`` plus the small numpy helpers in this package (direct-stiffness
solve, region selection in `regions.py`).  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does.

Arrays are dense over the nx*ny*nz cells (cell index x + nx*(y + ny*z)),
material 0 is empty, units are SI.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

VXO_OK = 0
VXO_EUNSTABLE = -3
VXO_EOVERFLOW = -4


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("cte", C.c_double), ("mu_s", C.c_double), ("mu_d", C.c_double)]


class Params(C.Structure):
    _fields_ = [("voxel_size", C.c_double), ("gravity", C.c_double),
                ("zeta_bond", C.c_double), ("zeta_slow", C.c_double), ("zeta_col", C.c_double),
                ("temp_amp", C.c_double), ("temp_freq", C.c_double), ("temp_phase", C.c_double),
                ("dt_scale", C.c_double), ("origin", C.c_double * 3),
                ("floor_on", C.c_int32), ("self_collision_on", C.c_int32),
                ("contact_cap", C.c_int32), ("pad", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        # VX_ORACLE_LIB: another build of vx_oracle.c (the mutation check of
        # the pins loads deliberately broken copies this way)
        path = os.environ.get("VX_ORACLE_LIB") or _build.ensure_built()
        L = C.CDLL(path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.vxo_create.restype = P
        L.vxo_create.argtypes = [P, C.c_int, C.c_int, C.c_int, P, C.c_int, P]
        L.vxo_destroy.argtypes = [P]
        for n in ("vxo_set_fixed",):
            getattr(L, n).argtypes = [P, P]
        L.vxo_set_forces.argtypes = [P, P]
        L.vxo_set_actuation.argtypes = [P, P, P]
        L.vxo_set_velocity.argtypes = [P, P]
        L.vxo_step.argtypes = [P, C.c_longlong]
        L.vxo_read_state.argtypes = [P, P, P, P, P]
        L.vxo_write_state.argtypes = [P, P, P, P, P]
        L.vxo_read_flags.argtypes = [P, P, P]
        L.vxo_dt.restype = C.c_double
        L.vxo_dt.argtypes = [P]
        L.vxo_time.restype = C.c_double
        L.vxo_time.argtypes = [P]
        L.vxo_num_voxels.argtypes = [P]
        L.vxo_num_bonds.argtypes = [P]
        L.vxo_last_error.restype = C.c_char_p
        L.vxo_last_error.argtypes = [P]
        L.vxo_set_rebuild_every_step.argtypes = [P, C.c_int]
        L.vxo_rebuilds.restype = C.c_longlong
        L.vxo_rebuilds.argtypes = [P]
        L.vxo_candidates.argtypes = [P, P, P, C.c_int]
        L.vxo_energy.argtypes = [P, dp]
        L.vxo_bond_results.argtypes = [P, P, P, P, P]
        L.vxo_set_channels.argtypes = [P, P, C.c_int, P, C.c_int, P]
        L.vxo_channel_value.restype = C.c_double
        L.vxo_channel_value.argtypes = [P, C.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_palette(materials):
    """materials: list of dicts (index 0 must be the empty material)."""
    arr = (Material * len(materials))()
    for i, m in enumerate(materials):
        arr[i] = Material(m.get("E", 1.0), m.get("nu", 0.0), m.get("rho", 1.0), m.get("cte", 0.0),
                          m.get("mu_s", 0.0), m.get("mu_d", 0.0))
    return arr


def make_params(**kw):
    p = Params()
    p.voxel_size = kw.get("voxel_size", 1e-3)
    p.gravity = kw.get("gravity", 0.0)
    p.zeta_bond = kw.get("zeta_bond", 0.0)
    p.zeta_slow = kw.get("zeta_slow", 0.0)
    p.zeta_col = kw.get("zeta_col", 0.0)
    p.temp_amp = kw.get("temp_amp", 0.0)
    p.temp_freq = kw.get("temp_freq", 0.0)
    p.temp_phase = kw.get("temp_phase", 0.0)
    p.dt_scale = kw.get("dt_scale", 1.0)
    o = kw.get("origin", (0.0, 0.0, 0.0))
    p.origin[0], p.origin[1], p.origin[2] = o
    p.floor_on = int(kw.get("floor_on", 0))
    p.self_collision_on = int(kw.get("self_collision_on", 0))
    p.contact_cap = int(kw.get("contact_cap", 32))
    return p


WAVEFORMS = {"sine": 0, "triangle": 1, "square": 2}


class Channel(C.Structure):
    _fields_ = [("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double), ("offset", C.c_double),
                ("waveform", C.c_int32), ("pad", C.c_int32)]


def make_channels(channels):
    """ctypes array of channel dicts {amp, freq, phase, offset, waveform}."""
    arr = (Channel * max(len(channels), 1))()
    for i, c in enumerate(channels):
        arr[i].amp = float(c.get("amp", 0.0))
        arr[i].freq = float(c.get("freq", 0.0))
        arr[i].phase = float(c.get("phase", 0.0))
        arr[i].offset = float(c.get("offset", 0.0))
        wf = c.get("waveform", "sine")
        arr[i].waveform = WAVEFORMS[wf] if isinstance(wf, str) else int(wf)
    return arr


def channel_value(channel, t):
    """The oracle's temperature of one channel dict at time t."""
    arr = make_channels([channel])
    return lib().vxo_channel_value(C.cast(arr, C.c_void_p), float(t))


class Sim:
    """One oracle simulation.  ``grid`` is a uint8 array of shape (nz, ny, nx)
    (so that a C-order flatten gives x fastest)."""

    def __init__(self, grid, materials, **params):
        L = lib()
        g = np.ascontiguousarray(grid, dtype=np.uint8)
        assert g.ndim == 3
        self.nz, self.ny, self.nx = g.shape
        self.grid = g
        self.ncell = g.size
        self._pal = make_palette(materials)
        self._prm = make_params(**params)
        self.voxel_size = self._prm.voxel_size
        h = L.vxo_create(_ptr(g), self.nx, self.ny, self.nz, C.cast(self._pal, C.c_void_p),
                         len(materials), C.cast(C.pointer(self._prm), C.c_void_p))
        if not h:
            raise ValueError("oracle rejected the lattice or materials")
        self.h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().vxo_destroy(h)
            self.h = None

    # setters (dense per-cell arrays)
    def set_fixed(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        assert m.size == self.ncell
        lib().vxo_set_fixed(self.h, _ptr(m))

    def set_forces(self, F):
        f = np.ascontiguousarray(F, dtype=np.float64).reshape(self.ncell, 3)
        lib().vxo_set_forces(self.h, _ptr(f))

    def set_actuation(self, amp=None, phase=None):
        a = None if amp is None else np.ascontiguousarray(amp, dtype=np.float64).reshape(-1)
        p = None if phase is None else np.ascontiguousarray(phase, dtype=np.float64).reshape(-1)
        lib().vxo_set_actuation(self.h, _ptr(a), _ptr(p))

    def set_velocity(self, v):
        vv = np.ascontiguousarray(v, dtype=np.float64).reshape(self.ncell, 3)
        lib().vxo_set_velocity(self.h, _ptr(vv))

    def set_channels(self, channels, mat_channel=None, cell_channel=None):
        """Named actuation channels: a list of dicts {amp, freq, phase,
        offset, waveform}; mat_channel gives each palette entry's channel
        (-1 none), cell_channel each cell's (-1: its material's)."""
        self._chan = make_channels(channels)
        mc = None if mat_channel is None else np.ascontiguousarray(mat_channel, dtype=np.int32)
        cc = None if cell_channel is None else np.ascontiguousarray(cell_channel, dtype=np.int32).reshape(-1)
        rc = lib().vxo_set_channels(self.h, C.cast(self._chan, C.c_void_p), len(channels), _ptr(mc),
                                    0 if mc is None else mc.size, _ptr(cc))
        if rc != 0:
            raise ValueError("oracle rejected the channels")

    def set_rebuild_every_step(self, on=True):
        lib().vxo_set_rebuild_every_step(self.h, int(on))

    def step(self, n=1):
        return lib().vxo_step(self.h, int(n))

    @property
    def dt(self):
        return lib().vxo_dt(self.h)

    @property
    def time(self):
        return lib().vxo_time(self.h)

    @property
    def num_voxels(self):
        return lib().vxo_num_voxels(self.h)

    @property
    def num_bonds(self):
        return lib().vxo_num_bonds(self.h)

    @property
    def rebuilds(self):
        return lib().vxo_rebuilds(self.h)

    def last_error(self):
        return lib().vxo_last_error(self.h).decode()

    def read_state(self):
        n = self.ncell
        u = np.empty((n, 3)); q = np.empty((n, 4)); v = np.empty((n, 3)); w = np.empty((n, 3))
        lib().vxo_read_state(self.h, _ptr(u), _ptr(q), _ptr(v), _ptr(w))
        return {"u": u, "q": q, "v": v, "w": w}

    def write_state(self, u=None, q=None, v=None, w=None):
        conv = lambda a, k: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.ncell, k)
        u, q, v, w = conv(u, 3), conv(q, 4), conv(v, 3), conv(w, 3)
        lib().vxo_write_state(self.h, _ptr(u), _ptr(q), _ptr(v), _ptr(w))

    def read_flags(self):
        st = np.empty(self.ncell, np.uint8); su = np.empty(self.ncell, np.uint8)
        lib().vxo_read_flags(self.h, _ptr(st), _ptr(su))
        return {"static": st, "surface": su}

    def candidates(self):
        n = lib().vxo_candidates(self.h, None, None, 0)
        a = np.empty(max(n, 1), np.int32); b = np.empty(max(n, 1), np.int32)
        lib().vxo_candidates(self.h, _ptr(a), _ptr(b), n)
        return set(zip(a[:n].tolist(), b[:n].tolist()))

    def energy(self):
        out = (C.c_double * 12)()
        lib().vxo_energy(self.h, out)
        o = list(out)
        return {"ke": o[0], "elastic": o[1], "gravity": o[2], "floor": o[3], "power": o[4],
                "P": np.array(o[6:9]), "L": np.array(o[9:12])}

    def bond_results(self):
        n = self.num_bonds
        c1 = np.empty(n, np.int32); c2 = np.empty(n, np.int32); ax = np.empty(n, np.int32)
        r = np.empty((n, 9))
        lib().vxo_bond_results(self.h, _ptr(c1), _ptr(c2), _ptr(ax), _ptr(r))
        return c1, c2, ax, r
