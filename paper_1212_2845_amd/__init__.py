"""voxsim: MI355X (gfx950) explicit time step of a heterogeneous voxel lattice.

Thin ctypes binding over the C ABI of ``libvoxsim.so`` (declared in
``include/voxsim.h``).  Every step of the simulation runs in the library's HIP
kernels; this module only marshals arguments and lets PyTorch own the device
workspace and supply the stream.  There is no fallback: if the shared library
is missing the import of :func:`lib` raises.

Method: Hiller & Lipson, "Dynamic Simulation of Soft Heterogeneous Objects"
(arXiv 1212.2845), section "Physics Engine".
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvoxsim.so")

VX_OK = 0
VX_EINVAL = -1
VX_EDEVICE = -2
VX_EUNSTABLE = -3
VX_EOVERFLOW = -4
VX_ESTATE = -5
VX_ENOMEM = -6

KERNEL_FUSED = 0
KERNEL_SPLIT = 1

EXPORTED = ["vx_create", "vx_workspace_bytes", "vx_bind_workspace", "vx_set_fixed", "vx_set_forces",
            "vx_fixed_region", "vx_forced_region", "vx_set_actuation", "vx_set_velocity", "vx_step",
            "vx_read_state", "vx_write_state", "vx_read_flags", "vx_get_dt", "vx_get_time",
            "vx_counters", "vx_candidates", "vx_set_kernel", "vx_set_fused_tile", "vx_get_fused_tile",
            "vx_autotune", "vx_time_kernel", "vx_destroy", "vx_last_error",
            "vx_step_enqueue", "vx_status", "vx_probe", "vx_set_collision_mode", "vx_static_workspace_bytes",
            "vx_static_solve", "vx_static_solve_noalloc", "vx_energy", "vx_energy_enqueue", "vx_set_channels", "vx_grad_channels", "vx_set_stiffness", "vx_set_density", "vx_grad_workspace_bytes", "vx_grad_bind", "vx_grad_forward",
            "vx_grad_backward",
            "vx_batch_create", "vx_batch_workspace_bytes", "vx_batch_bind_workspace", "vx_batch_step",
            "vx_batch_read_state", "vx_batch_write_state", "vx_batch_get_dt", "vx_batch_counters",
            "vx_batch_set_launch", "vx_batch_autotune", "vx_batch_destroy", "vx_batch_last_error",
            "vx_batch_candidates", "vx_batch_contact_counters", "vx_batch_set_tile_rule", "vx_batch_get_tile"]

# state words, in the order vx_probe numbers them
WORDS = ["ux", "uy", "uz", "qw", "qx", "qy", "qz", "px", "py", "pz", "lx", "ly", "lz"]
FUSED_SHAPES = [(32, 8), (64, 4), (16, 16), (50, 5), (20, 12)]


class VoxsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("voxsim error %d: %s" % (code, msg))
        self.code = code


class Material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("cte", C.c_double), ("mu_s", C.c_double), ("mu_d", C.c_double)]


WAVEFORMS = {"sine": 0, "triangle": 1, "square": 2}
MAX_CHANNELS = 8


class Channel(C.Structure):
    _fields_ = [("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double), ("offset", C.c_double),
                ("waveform", C.c_int32), ("reserved", C.c_int32)]


class Object(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("reserved", C.c_int32), ("origin", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("voxel_size", C.c_double), ("gravity", C.c_double),
                ("zeta_bond", C.c_double), ("zeta_slow", C.c_double), ("zeta_col", C.c_double),
                ("temp_amp", C.c_double), ("temp_freq", C.c_double), ("temp_phase", C.c_double),
                ("dt_scale", C.c_double), ("origin", C.c_double * 3),
                ("floor_on", C.c_int32), ("self_collision_on", C.c_int32),
                ("contact_cap", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib():
    """Load libvoxsim.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvoxsim.so not found at %s; build it with "
                          "python -m paper_1212_2845_amd.build" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname as ROCm's; load
    # it first so that the library and torch share one runtime (device
    # pointers from torch tensors are then valid in the library's calls)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, i64, u64 = C.c_int32, C.c_int64, C.c_uint64
    L.vx_create.argtypes = [P, i32, i32, i32, P, i32, P, i32, P, C.POINTER(P)]
    L.vx_workspace_bytes.argtypes = [P, C.POINTER(u64)]
    L.vx_bind_workspace.argtypes = [P, P, u64]
    L.vx_set_fixed.argtypes = [P, P]
    L.vx_set_forces.argtypes = [P, P]
    L.vx_fixed_region.argtypes = [P, P, P]
    L.vx_forced_region.argtypes = [P, P, P, P]
    L.vx_set_actuation.argtypes = [P, P, P]
    L.vx_set_velocity.argtypes = [P, P]
    L.vx_step.argtypes = [P, i64]
    L.vx_read_state.argtypes = [P, P, P, P, P]
    L.vx_write_state.argtypes = [P, P, P, P, P]
    L.vx_read_flags.argtypes = [P, P, P]
    L.vx_get_dt.argtypes = [P, C.POINTER(C.c_double)]
    L.vx_get_time.argtypes = [P, C.POINTER(C.c_double)]
    L.vx_counters.argtypes = [P, C.POINTER(C.c_int64)]
    L.vx_candidates.argtypes = [P, P, P, i32, C.POINTER(i32)]
    L.vx_set_kernel.argtypes = [P, i32]
    L.vx_set_fused_tile.argtypes = [P, i32, i32]
    pi32 = C.POINTER(i32)
    L.vx_get_fused_tile.argtypes = [P, pi32, pi32, pi32, pi32]
    L.vx_autotune.argtypes = [P, i32, pi32, pi32]
    L.vx_time_kernel.argtypes = [P, i32, C.POINTER(C.c_double)]
    L.vx_energy.argtypes = [P, C.POINTER(C.c_double)]
    L.vx_energy_enqueue.argtypes = [P, P]
    L.vx_step_enqueue.argtypes = [P, i64]
    L.vx_status.argtypes = [P]
    L.vx_probe.argtypes = [P, P, i32, i32, P]
    L.vx_set_collision_mode.argtypes = [P, i32, i32]
    L.vx_static_workspace_bytes.argtypes = [P, C.POINTER(C.c_uint64)]
    L.vx_static_solve.argtypes = [P, P, C.c_uint64, P, C.c_double, i32, P, P, C.POINTER(i32),
                                  C.POINTER(C.c_double)]
    L.vx_static_solve_noalloc.argtypes = [P, P, C.c_double, i32, P, P, C.POINTER(i32), C.POINTER(C.c_double)]
    L.vx_set_channels.argtypes = [P, P, i32, P, P]
    L.vx_grad_channels.argtypes = [P, P, P]
    L.vx_set_stiffness.argtypes = [P, P]
    L.vx_set_density.argtypes = [P, P]
    L.vx_grad_workspace_bytes.argtypes = [P, i64, i32, C.POINTER(u64)]
    L.vx_grad_bind.argtypes = [P, P, u64, i64, i32]
    L.vx_grad_forward.argtypes = [P, i64]
    L.vx_grad_backward.argtypes = [P] + [P] * 12
    L.vx_destroy.argtypes = [P]
    L.vx_last_error.argtypes = [P]
    L.vx_last_error.restype = C.c_char_p
    L.vx_batch_create.argtypes = [P, i32, P, i32, P, i32, P, C.POINTER(P)]
    L.vx_batch_workspace_bytes.argtypes = [P, C.POINTER(u64)]
    L.vx_batch_bind_workspace.argtypes = [P, P, u64]
    L.vx_batch_step.argtypes = [P, i64]
    L.vx_batch_read_state.argtypes = [P, i32, P, P, P, P]
    L.vx_batch_write_state.argtypes = [P, i32, P, P, P, P]
    L.vx_batch_get_dt.argtypes = [P, i32, C.POINTER(C.c_double)]
    L.vx_batch_counters.argtypes = [P, C.POINTER(C.c_int64)]
    L.vx_batch_set_launch.argtypes = [P, i32, i32]
    L.vx_batch_autotune.argtypes = [P, i32, pi32]
    L.vx_batch_set_tile_rule.argtypes = [P, i32]
    L.vx_batch_get_tile.argtypes = [P, i32, pi32]
    L.vx_batch_candidates.argtypes = [P, P, P, P, P, i32, pi32]
    L.vx_batch_contact_counters.argtypes = [P, C.POINTER(C.c_int64)]
    L.vx_batch_destroy.argtypes = [P]
    L.vx_batch_last_error.argtypes = [P]
    L.vx_batch_last_error.restype = C.c_char_p
    for n in EXPORTED:
        if n not in ("vx_last_error", "vx_batch_last_error"):
            getattr(L, n).restype = C.c_int
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_palette(materials):
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
    p.reserved = 0
    return p


class Sim:
    """One lattice simulation on the GPU.

    ``grid`` is a uint8 array of shape (nz, ny, nx) (a C-order flatten gives the
    library's cell order, x fastest); ``materials`` a list of dicts with keys
    E, nu, rho, cte, mu_s, mu_d (index 0 = empty); ``precision`` 32 or 64.
    The device workspace is a torch uint8 tensor allocated on first use.
    """

    def __init__(self, grid, materials, precision=64, device=None, stream=None, kernel=KERNEL_FUSED,
                 **params):
        L = lib()
        g = np.ascontiguousarray(grid, dtype=np.uint8)
        if g.ndim != 3:
            raise ValueError("grid must be 3-D (nz, ny, nx)")
        self.nz, self.ny, self.nx = g.shape
        self.ncell = g.size
        self.grid = g
        self.precision = int(precision)
        self._pal = make_palette(materials)
        self.n_mat = len(materials)
        self._prm = make_params(**params)
        self._device = device
        self._stream = stream
        self._ws = None
        h = C.c_void_p()
        rc = L.vx_create(_ptr(g), self.nx, self.ny, self.nz, C.cast(self._pal, C.c_void_p), len(materials),
                         C.cast(C.pointer(self._prm), C.c_void_p), self.precision, self._stream_ptr(),
                         C.byref(h))
        if rc != VX_OK:
            raise VoxsimError(rc, "vx_create rejected the lattice, palette or parameters")
        self.h = h
        self._check(L.vx_set_kernel(self.h, int(kernel)))

    # -- plumbing -----------------------------------------------------------
    def _stream_ptr(self):
        if self._stream is not None:
            return C.c_void_p(int(self._stream))
        return None

    def _check(self, rc):
        if rc != VX_OK:
            raise VoxsimError(rc, lib().vx_last_error(self.h).decode())

    def workspace_bytes(self):
        n = C.c_uint64()
        self._check(lib().vx_workspace_bytes(self.h, C.byref(n)))
        return n.value

    def bind(self):
        """Allocate the device workspace with torch and bind it."""
        if self._ws is not None:
            return
        import torch
        dev = self._device or torch.device("cuda", torch.cuda.current_device())
        nbytes = self.workspace_bytes()
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self._check(lib().vx_bind_workspace(self.h, C.c_void_p(self._ws.data_ptr()), nbytes))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.vx_destroy(h)
            self.h = None

    # -- setters --------------------------------------------------------------
    def set_kernel(self, kind):
        self._check(lib().vx_set_kernel(self.h, int(kind)))

    def set_fused_tile(self, shape=-1, zc=0):
        self._check(lib().vx_set_fused_tile(self.h, int(shape), int(zc)))

    def fused_tile(self):
        v = [C.c_int32() for _ in range(4)]
        self._check(lib().vx_get_fused_tile(self.h, *[C.byref(x) for x in v]))
        return {"shape": v[0].value, "tx": v[1].value, "ty": v[2].value, "zc": v[3].value}

    def time_kernel(self, iters=20):
        """Average ms of one step-kernel launch (dry runs, state unchanged)."""
        self.bind()
        ms = C.c_double()
        self._check(lib().vx_time_kernel(self.h, int(iters), C.byref(ms)))
        return ms.value

    def autotune(self, iters=5):
        self.bind()
        sh = C.c_int32(); zc = C.c_int32()
        self._check(lib().vx_autotune(self.h, int(iters), C.byref(sh), C.byref(zc)))
        return self.fused_tile()

    def set_fixed(self, mask):
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        assert m.size == self.ncell
        self._check(lib().vx_set_fixed(self.h, _ptr(m)))

    def set_forces(self, F):
        f = np.ascontiguousarray(F, dtype=np.float64).reshape(self.ncell, 3)
        self._check(lib().vx_set_forces(self.h, _ptr(f)))

    def fixed_region(self, loc, size):
        a = np.asarray(loc, np.float64); b = np.asarray(size, np.float64)
        self._check(lib().vx_fixed_region(self.h, _ptr(a), _ptr(b)))

    def forced_region(self, loc, size, force):
        a = np.asarray(loc, np.float64); b = np.asarray(size, np.float64); f = np.asarray(force, np.float64)
        self._check(lib().vx_forced_region(self.h, _ptr(a), _ptr(b), _ptr(f)))

    def set_actuation(self, amp=None, phase=None):
        a = None if amp is None else np.ascontiguousarray(amp, dtype=np.float64).reshape(-1)
        p = None if phase is None else np.ascontiguousarray(phase, dtype=np.float64).reshape(-1)
        self._check(lib().vx_set_actuation(self.h, _ptr(a), _ptr(p)))

    def set_velocity(self, v):
        vv = np.ascontiguousarray(v, dtype=np.float64).reshape(self.ncell, 3)
        self._check(lib().vx_set_velocity(self.h, _ptr(vv)))

    # -- stepping and reading ----------------------------------------------------
    def step(self, n=1):
        self.bind()
        self._check(lib().vx_step(self.h, int(n)))

    def step_rc(self, n=1):
        """Step and return the status code instead of raising."""
        self.bind()
        return lib().vx_step(self.h, int(n))

    def step_enqueue(self, n=1):
        """Enqueue n steps without waiting (capturable into a HIP graph)."""
        self._check(lib().vx_step_enqueue(self.h, int(n)))

    def status(self):
        """Wait for the stream; raise on a non-finite state or overflow."""
        self._check(lib().vx_status(self.h))

    def static_solve(self, F, rel_tol=1e-10, max_iter=200000):
        """Linear direct-stiffness solution under the load F (ncell x 3 N)
        with the clamped voxels of set_fixed (see vx_static_solve).  Returns
        u and theta (ncell x 3), the iteration count and the true relative
        residual."""
        import torch
        self.bind()
        n = C.c_uint64()
        self._check(lib().vx_static_workspace_bytes(self.h, C.byref(n)))
        work = torch.empty(n.value, dtype=torch.uint8, device=self._ws.device)
        f = np.ascontiguousarray(F, dtype=np.float64).reshape(self.ncell, 3)
        u = np.empty((self.ncell, 3)); th = np.empty((self.ncell, 3))
        it = C.c_int32(); res = C.c_double()
        self._check(lib().vx_static_solve(self.h, C.c_void_p(work.data_ptr()), n.value, _ptr(f), float(rel_tol),
                                          int(max_iter), _ptr(u), _ptr(th), C.byref(it), C.byref(res)))
        return {"u": u, "theta": th, "iters": it.value, "rel_residual": res.value}

    def static_solve_noalloc(self, F, rel_tol=1e-10, max_iter=200000):
        """static_solve through vx_static_solve_noalloc: the same solve in the
        library's fixed device scratch, with no workspace allocated."""
        self.bind()
        f = np.ascontiguousarray(F, dtype=np.float64).reshape(self.ncell, 3)
        u = np.empty((self.ncell, 3)); th = np.empty((self.ncell, 3))
        it = C.c_int32(); res = C.c_double()
        self._check(lib().vx_static_solve_noalloc(self.h, _ptr(f), float(rel_tol), int(max_iter), _ptr(u), _ptr(th),
                                                  C.byref(it), C.byref(res)))
        return {"u": u, "theta": th, "iters": it.value, "rel_residual": res.value}

    def set_channels(self, channels, mat_channel=None, cell_channel=None):
        """Named actuation channels (see vx_set_channels): a list of dicts
        {amp, freq, phase, offset, waveform ('sine' | 'triangle' |
        'square')}; mat_channel gives each palette entry's channel (-1:
        none), cell_channel each cell's (-1: its material's)."""
        n = len(channels)
        arr = (Channel * max(n, 1))()
        for i, c in enumerate(channels):
            arr[i].amp = float(c.get("amp", 0.0))
            arr[i].freq = float(c.get("freq", 0.0))
            arr[i].phase = float(c.get("phase", 0.0))
            arr[i].offset = float(c.get("offset", 0.0))
            wf = c.get("waveform", "sine")
            arr[i].waveform = WAVEFORMS[wf] if isinstance(wf, str) else int(wf)
            arr[i].reserved = 0
        mc = None
        if mat_channel is not None:
            mc = np.ascontiguousarray(mat_channel, dtype=np.int32)
            assert mc.size == self.n_mat
        cc = None if cell_channel is None else np.ascontiguousarray(cell_channel, dtype=np.int32).reshape(-1)
        if cc is not None:
            assert cc.size == self.ncell
        self._check(lib().vx_set_channels(self.h, C.cast(arr, C.c_void_p), n, _ptr(mc), _ptr(cc)))
        self._n_chan = n

    def grad_channels(self):
        """Per-channel dL/dphase and dL/damp of the last grad_backward."""
        n = getattr(self, "_n_chan", 0)
        gp = np.zeros(max(n, 1)); ga = np.zeros(max(n, 1))
        self._check(lib().vx_grad_channels(self.h, _ptr(gp), _ptr(ga)))
        return {"phase": gp[:n], "amp": ga[:n]}

    def set_collision_mode(self, all_voxels=False, every_step=False):
        """Self-collision scheme (see vx_set_collision_mode): candidates from
        all filled voxels or the surface only; rebuilt every step or by the
        horizon rule."""
        self._check(lib().vx_set_collision_mode(self.h, int(bool(all_voxels)), int(bool(every_step))))

    def probe(self, cells, word, out):
        """Enqueue a copy of state word ``word`` (0..12, see WORDS) of the
        cells in the int32 device tensor ``cells`` into the device tensor
        ``out`` (float32 or float64 as the state) without waiting."""
        import torch
        assert cells.is_cuda and out.is_cuda and cells.dtype == torch.int32
        assert out.dtype == (torch.float64 if self.precision == 64 else torch.float32)
        assert cells.is_contiguous() and out.is_contiguous() and out.numel() >= cells.numel()
        self.bind()
        self._check(lib().vx_probe(self.h, C.c_void_p(cells.data_ptr()), int(cells.numel()), int(word),
                                   C.c_void_p(out.data_ptr())))

    @property
    def dt(self):
        d = C.c_double()
        self._check(lib().vx_get_dt(self.h, C.byref(d)))
        return d.value

    @property
    def time(self):
        d = C.c_double()
        self._check(lib().vx_get_time(self.h, C.byref(d)))
        return d.value

    def counters(self):
        out = (C.c_int64 * 4)()
        self._check(lib().vx_counters(self.h, out))
        return {"steps": out[0], "rebuilds": out[1], "pairs": out[2], "voxels": out[3]}

    def read_state(self):
        n = self.ncell
        u = np.empty((n, 3)); q = np.empty((n, 4)); v = np.empty((n, 3)); w = np.empty((n, 3))
        self._check(lib().vx_read_state(self.h, _ptr(u), _ptr(q), _ptr(v), _ptr(w)))
        return {"u": u, "q": q, "v": v, "w": w}

    def write_state(self, u=None, q=None, v=None, w=None):
        conv = lambda a, k: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.ncell, k)
        u, q, v, w = conv(u, 3), conv(q, 4), conv(v, 3), conv(w, 3)
        self._check(lib().vx_write_state(self.h, _ptr(u), _ptr(q), _ptr(v), _ptr(w)))

    def energy(self):
        """Energies and momenta of the current state (see vx_energy)."""
        self.bind()
        out = (C.c_double * 10)()
        self._check(lib().vx_energy(self.h, out))
        v = list(out)
        return {"kinetic": v[0], "elastic": v[1], "gravity": v[2], "floor": v[3], "momentum": v[4:7],
                "angular_momentum": v[7:10]}

    ENERGY_KEYS = ("kinetic", "elastic", "gravity", "floor", "Px", "Py", "Pz", "Lx", "Ly", "Lz")

    def energy_enqueue(self, out):
        """Enqueue the vx_energy sums of the current state into ``out``, a
        float64 device tensor of at least 10 elements, without waiting."""
        import torch
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= 10
        self.bind()
        self._check(lib().vx_energy_enqueue(self.h, C.c_void_p(out.data_ptr())))

    def energy_record(self, steps, every=1, device=None):
        """Run ``steps`` steps (a multiple of ``every``) with the energies of
        the state before the first step and after every ``every`` steps
        recorded on the device; one wait at the end.  Returns a float64
        device tensor of shape (steps // every + 1, 10), columns as
        ENERGY_KEYS."""
        import torch
        assert steps >= 0 and every >= 1 and steps % every == 0
        self.bind()
        rec = torch.empty((steps // every + 1, 10), dtype=torch.float64, device=device or "cuda")
        self.energy_enqueue(rec[0])
        for k in range(1, rec.shape[0]):
            self._check(lib().vx_step_enqueue(self.h, every))
            self.energy_enqueue(rec[k])
        self.status()
        return rec

    def read_flags(self):
        st = np.empty(self.ncell, np.uint8); su = np.empty(self.ncell, np.uint8)
        self._check(lib().vx_read_flags(self.h, _ptr(st), _ptr(su)))
        return {"static": st, "surface": su}

    def candidates(self):
        n = C.c_int32()
        self._check(lib().vx_candidates(self.h, None, None, 0, C.byref(n)))
        k = n.value
        a = np.empty(max(k, 1), np.int32); b = np.empty(max(k, 1), np.int32)
        self._check(lib().vx_candidates(self.h, _ptr(a), _ptr(b), k, C.byref(n)))
        return set(zip(a[:k].tolist(), b[:k].tolist()))


    # -- parameter mode and differentiable rollouts --------------------------
    def set_stiffness(self, E):
        """Per-voxel elastic modulus (ncell values; None returns to the palette)."""
        e = None if E is None else np.ascontiguousarray(E, dtype=np.float64).reshape(-1)
        if e is not None:
            assert e.size == self.ncell
        self._check(lib().vx_set_stiffness(self.h, _ptr(e)))

    def set_density(self, rho):
        """Per-voxel density (ncell values; None returns to the palette)."""
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        if r is not None:
            assert r.size == self.ncell
        self._check(lib().vx_set_density(self.h, _ptr(r)))

    def grad_workspace_bytes(self, max_steps, K):
        """Bytes vx_grad_bind needs for rollouts of up to max_steps steps
        with a checkpoint every K steps (K = 1: the full tape)."""
        n = C.c_uint64()
        self._check(lib().vx_grad_workspace_bytes(self.h, int(max_steps), int(K), C.byref(n)))
        return n.value

    def grad_bind(self, max_steps, K):
        """Allocate (torch) and bind the gradient workspace for rollouts of up
        to max_steps steps with a checkpoint every K steps."""
        import torch
        self.bind()
        n = C.c_uint64()
        self._check(lib().vx_grad_workspace_bytes(self.h, int(max_steps), int(K), C.byref(n)))
        if getattr(self, "_gws", None) is None or self._gws.numel() < n.value:
            self._gws = None
            self._gws = torch.empty(n.value, dtype=torch.uint8, device=self._ws.device)
        self._check(lib().vx_grad_bind(self.h, C.c_void_p(self._gws.data_ptr()), n.value, int(max_steps), int(K)))
        return n.value

    def grad_forward(self, n):
        self._check(lib().vx_grad_forward(self.h, int(n)))

    def grad_backward(self, dL_du=None, dL_dq=None, dL_dv=None, dL_dw=None, initial_state=True):
        """Gradients of a function of the final state (adjoints given per
        cell, None = 0) w.r.t. the moduli, the densities, the per-voxel
        actuation phase and amplitude, and (with initial_state) the
        rollout's initial state (keys u0, q0, v0, w0)."""
        n = self.ncell
        conv = lambda a, k: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(n, k)
        du, dq, dv, dw = conv(dL_du, 3), conv(dL_dq, 4), conv(dL_dv, 3), conv(dL_dw, 3)
        out = {"E": np.empty(n), "rho": np.empty(n), "phase": np.empty(n), "amp": np.empty(n)}
        if initial_state:
            out.update({"u0": np.empty((n, 3)), "q0": np.empty((n, 4)), "v0": np.empty((n, 3)),
                        "w0": np.empty((n, 3))})
        self._check(lib().vx_grad_backward(self.h, _ptr(du), _ptr(dq), _ptr(dv), _ptr(dw), _ptr(out["E"]),
                                           _ptr(out["rho"]), _ptr(out["phase"]), _ptr(out["amp"]),
                                           _ptr(out.get("u0")), _ptr(out.get("q0")), _ptr(out.get("v0")),
                                           _ptr(out.get("w0"))))
        return out


def _rollout_fn():
    import torch

    class RolloutFn(torch.autograd.Function):
        """Final displacement and velocity (ncell x 3 each, float64, CPU) of an
        n-step rollout from the Sim's current state, differentiable w.r.t. the
        per-voxel modulus E, density rho, actuation phase and actuation
        amplitude amp (ncell each, on any device).  Gradients come back on
        each input's device and in its dtype."""

        @staticmethod
        def forward(ctx, E, rho, phase, amp, sim, n):
            sim.set_stiffness(E.detach().cpu().numpy())
            sim.set_density(rho.detach().cpu().numpy())
            sim.set_actuation(amp.detach().cpu().numpy(), phase.detach().cpu().numpy())
            sim.grad_forward(n)
            st = sim.read_state()
            ctx.sim = sim
            ctx.like = [(t.device, t.dtype) for t in (E, rho, phase, amp)]
            return torch.from_numpy(st["u"]), torch.from_numpy(st["v"])

        @staticmethod
        def backward(ctx, gu, gv):
            g = ctx.sim.grad_backward(dL_du=gu.detach().cpu().numpy(), dL_dv=gv.detach().cpu().numpy(),
                                      initial_state=False)
            out = [torch.from_numpy(g[k]).to(device=d, dtype=t)
                   for k, (d, t) in zip(("E", "rho", "phase", "amp"), ctx.like)]
            return tuple(out) + (None, None)

    return RolloutFn


def rollout(sim, E, rho, phase, amp, n):
    """(u, v) after n steps from sim's current state; differentiable in E,
    rho, phase and amp (torch tensors of ncell values; amp may also be an
    array, then held fixed) through the library's reverse run (sim needs
    grad_bind first)."""
    import torch
    if not isinstance(amp, torch.Tensor):
        amp = torch.as_tensor(np.asarray(amp, dtype=np.float64))
    return _rollout_fn().apply(E, rho, phase, amp, sim, n)


def from_workload(w, precision=64, kernel=KERNEL_FUSED, stream=None):
    """Build a Sim from a workload dict of the seeded input generators."""
    s = Sim(w["grid"], w["materials"], precision=precision, kernel=kernel, stream=stream, **w["params"])
    if w.get("fixed") is not None:
        s.set_fixed(w["fixed"])
    if w.get("forces") is not None:
        s.set_forces(w["forces"])
    if w.get("amp") is not None or w.get("phase") is not None:
        s.set_actuation(w.get("amp"), w.get("phase"))
    if w.get("velocity") is not None:
        s.set_velocity(w["velocity"])
    return s


class Batch:
    """Many independent objects (same palette and parameters) stepped by one
    persistent launch.  ``grids`` is a list of uint8 arrays (nz, ny, nx);
    ``origins`` an optional list of (x, y, z) lower-corner positions."""

    def __init__(self, grids, materials, precision=32, device=None, stream=None, origins=None, **params):
        L = lib()
        self._grids = [np.ascontiguousarray(g, dtype=np.uint8) for g in grids]
        n = len(self._grids)
        objs = (Object * n)()
        for i, g in enumerate(self._grids):
            objs[i].grid = g.ctypes.data_as(C.c_void_p)
            objs[i].nz, objs[i].ny, objs[i].nx = g.shape
            objs[i].reserved = 0
            o = origins[i] if origins is not None else params.get("origin", (0.0, 0.0, 0.0))
            objs[i].origin[0], objs[i].origin[1], objs[i].origin[2] = o
        self._objs = objs
        self._pal = make_palette(materials)
        self._prm = make_params(**params)
        self.precision = int(precision)
        self._device = device
        self._stream = stream
        self._ws = None
        h = C.c_void_p()
        rc = L.vx_batch_create(C.cast(objs, C.c_void_p), n, C.cast(self._pal, C.c_void_p), len(materials),
                               C.cast(C.pointer(self._prm), C.c_void_p), self.precision,
                               None if stream is None else C.c_void_p(int(stream)), C.byref(h))
        if rc != VX_OK:
            raise VoxsimError(rc, "vx_batch_create rejected the objects, palette or parameters")
        self.h = h
        self.n = n

    def _check(self, rc):
        if rc != VX_OK:
            raise VoxsimError(rc, lib().vx_batch_last_error(self.h).decode())

    def bind(self):
        if self._ws is not None:
            return
        import torch
        dev = self._device or torch.device("cuda", torch.cuda.current_device())
        nb = C.c_uint64()
        self._check(lib().vx_batch_workspace_bytes(self.h, C.byref(nb)))
        self._ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        self._check(lib().vx_batch_bind_workspace(self.h, C.c_void_p(self._ws.data_ptr()), nb.value))

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.vx_batch_destroy(h)
            self.h = None

    def set_launch(self, n_workgroups=0, max_steps_per_launch=0):
        self._check(lib().vx_batch_set_launch(self.h, int(n_workgroups), int(max_steps_per_launch)))

    def autotune(self, steps=20):
        """Times each tile rule with candidate workgroup counts and keeps the
        fastest pair; returns the workgroup count (the rule: tile(i)[0])."""
        self.bind()
        nw = C.c_int32()
        self._check(lib().vx_batch_autotune(self.h, int(steps), C.byref(nw)))
        return nw.value

    def set_tile_rule(self, rule):
        """0: the widest rows; 1: rule 0's tiles across x with their widths
        evened out (differs for footprints over 64 cells wide)."""
        self._check(lib().vx_batch_set_tile_rule(self.h, int(rule)))

    def tile(self, i):
        """(rule in force, TX, TY) of object i."""
        out = (C.c_int32 * 3)()
        self._check(lib().vx_batch_get_tile(self.h, int(i), out))
        return out[0], out[1], out[2]

    def step(self, n=1):
        self.bind()
        self._check(lib().vx_batch_step(self.h, int(n)))

    def dt(self, i):
        d = C.c_double()
        self._check(lib().vx_batch_get_dt(self.h, int(i), C.byref(d)))
        return d.value

    def counters(self):
        out = (C.c_int64 * 4)()
        self._check(lib().vx_batch_counters(self.h, out))
        return {"steps": out[0], "objects": out[1], "cells": out[2], "voxels": out[3]}

    def candidates(self):
        """Contact candidate pairs ((obj_a, cell_a), (obj_b, cell_b)), each
        pair once (see vx_batch_candidates)."""
        n = C.c_int32()
        self._check(lib().vx_batch_candidates(self.h, None, None, None, None, 0, C.byref(n)))
        k = n.value
        oa, ca, ob, cb = (np.zeros(max(k, 1), np.int32) for _ in range(4))
        self._check(lib().vx_batch_candidates(self.h, _ptr(oa), _ptr(ca), _ptr(ob), _ptr(cb), k, C.byref(n)))
        return [((int(oa[i]), int(ca[i])), (int(ob[i]), int(cb[i]))) for i in range(k)]

    def contact_counters(self):
        out = (C.c_int64 * 3)()
        self._check(lib().vx_batch_contact_counters(self.h, out))
        return {"rebuilds": out[0], "pairs": out[1], "surface": out[2]}

    def read_state(self, i):
        self.bind()
        nc = self._grids[i].size
        u = np.empty((nc, 3)); q = np.empty((nc, 4)); v = np.empty((nc, 3)); w = np.empty((nc, 3))
        self._check(lib().vx_batch_read_state(self.h, int(i), _ptr(u), _ptr(q), _ptr(v), _ptr(w)))
        return {"u": u, "q": q, "v": v, "w": w}

    def write_state(self, i, u=None, q=None, v=None, w=None):
        self.bind()
        nc = self._grids[i].size
        conv = lambda a, k: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(nc, k)
        u, q, v, w = conv(u, 3), conv(q, 4), conv(v, 3), conv(w, 3)
        self._check(lib().vx_batch_write_state(self.h, int(i), _ptr(u), _ptr(q), _ptr(v), _ptr(w)))
