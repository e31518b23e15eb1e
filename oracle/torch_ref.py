"""Differentiable FP64 reference of the voxel-lattice step (test
infrastructure, like the rest of this package: only tests may use it).

The same method as vx_oracle.c, written a second time with plain PyTorch CPU
tensor operations in float64 so that torch.autograd gives reverse-mode
gradients of a rollout with respect to per-voxel modulus, density and
actuation phase and amplitude.  It is meant for tiny lattices (a few hundred
voxels, a few hundred steps).  It is pinned against the C oracle's
trajectory and against central differences of the C oracle
(tests/test_oracle_pins.py); it shares no code with the GPU library.

Steps, in the paper's order (Sec. 2-3):
  actuation: eps_v = cte_v dT_v(t_n), dT_v = A_v sin(2 pi f t_n + phi_v)
             (Eq. 39-40, per-voxel signal or the global one);
  bonds:     composite moduli (Eq. 1-2), beam constants (Eq. 8-12), voxel 1's
             co-rotational frame with the bond axis permuted onto x, the
             relative rotation vector, local end forces of the reduced
             stiffness (Eq. 13-24, z-force sign of the full matrix Eq. 7),
             applied with the opposite sign and rotated back, plus bond
             damping (Eq. 33-35);
  per voxel: sum of bond forces and moments (Eq. 25-26), external force,
             gravity, ground damping, floor penalty with normal damping,
             Coulomb friction (Eq. 36-38);
  integrate: P += F dt, u += P/m dt, phi += M dt, q <- normalise(dq(w dt) q)
             (Eq. 27-30 with the orientation as a unit quaternion).
"""
import math

import numpy as np
import torch

F64 = torch.float64


def _sum_sq(v):
    return (v * v).sum(-1)


def _quat_mul(a, b):
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


def _quat_conj(q):
    return q * torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64)


def _rot_matrix(q):
    """Columns of the rotation (body -> world) of unit quaternions, (n, 3, 3)
    with [:, :, k] the k-th body axis in the world."""
    w, x, y, z = q.unbind(-1)
    r = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)
    return r


def _log_rotvec(qr):
    """Rotation vector of unit quaternions on the short branch, 2 atan2(|v|, |w|)
    v/|v| (sign of w folded into v); a Taylor series of atan(t)/t near the
    identity keeps the value and its derivative defined at v = 0."""
    sg = torch.where(qr[..., 0] < 0, -1.0, 1.0).to(F64)
    w = sg * qr[..., 0]
    v = sg.unsqueeze(-1) * qr[..., 1:]
    s2 = _sum_sq(v)
    u = s2 / (w * w)
    small = u < 1e-2
    # atan(t)/t = sum (-1)^k u^k / (2k + 1), u = t^2
    ser = torch.zeros_like(u)
    for k in range(10, -1, -1):
        ser = ser * u + ((-1.0) ** k) / (2 * k + 1)
    k_small = 2.0 / w * ser
    s_safe = torch.sqrt(torch.where(small, torch.ones_like(s2), s2))
    k_big = 2.0 * torch.atan2(s_safe, w) / s_safe
    k = torch.where(small, k_small, k_big)
    return k.unsqueeze(-1) * v


def _exp_quat(r):
    """Unit quaternion of the rotation vector r: (cos |r|/2, sin(|r|/2) r/|r|)."""
    a2 = _sum_sq(r)
    small = a2 < 1e-4
    h2 = 0.25 * a2
    c_ser = torch.zeros_like(a2)
    s_ser = torch.zeros_like(a2)
    for k in range(8, -1, -1):
        c_ser = c_ser * h2 + ((-1.0) ** k) / math.factorial(2 * k)
        s_ser = s_ser * h2 + ((-1.0) ** k) / math.factorial(2 * k + 1)
    a_safe = torch.sqrt(torch.where(small, torch.ones_like(a2), a2))
    c = torch.where(small, c_ser, torch.cos(0.5 * a_safe))
    sk = torch.where(small, 0.5 * s_ser, torch.sin(0.5 * a_safe) / a_safe)   # sin(|r|/2) / |r|
    return torch.cat([c.unsqueeze(-1), sk.unsqueeze(-1) * r], -1)


class Lattice:
    """Static description of one workload (grid, palette, parameters,
    fixed and forced voxels, actuation), with per-voxel parameter defaults
    taken from the palette."""

    def __init__(self, w):
        g = np.asarray(w["grid"], np.uint8)
        self.nz, self.ny, self.nx = g.shape
        flat = g.reshape(-1)
        self.cells = np.nonzero(flat)[0]
        self.nvox = self.cells.size
        vid = -np.ones(flat.size, np.int64)
        vid[self.cells] = np.arange(self.nvox)
        p = w["params"]
        self.p = p
        self.l = float(p["voxel_size"])
        mats = w["materials"]
        mid = flat[self.cells]
        pal = lambda k: torch.tensor([mats[m][k] for m in mid], dtype=F64)
        self.E0, self.rho0 = pal("E"), pal("rho")
        self.nu, self.cte = pal("nu"), pal("cte")
        self.mu_s, self.mu_d = pal("mu_s"), pal("mu_d")
        x = self.cells % self.nx
        y = (self.cells // self.nx) % self.ny
        z = self.cells // (self.nx * self.ny)
        self.iz = torch.tensor(z, dtype=F64)
        self.rest = torch.tensor(np.stack([x, y, z], 1) + 0.5, dtype=F64) * self.l + torch.tensor(p["origin"],
                                                                                                  dtype=F64)
        # bonds per axis: voxel 1 = lower index along the axis
        self.bonds = []
        idx = np.stack([x, y, z], 1)
        dims = (self.nx, self.ny, self.nz)
        steps = (1, self.nx, self.nx * self.ny)
        for a in range(3):
            ok = idx[:, a] + 1 < dims[a]
            c1 = self.cells[ok]
            c2 = c1 + steps[a]
            has = flat[c2] > 0
            self.bonds.append((torch.tensor(vid[c1[has]]), torch.tensor(vid[c2[has]])))
        n = self.nvox
        fixed = w.get("fixed")
        self.fixed = torch.tensor(np.asarray(fixed).reshape(-1)[self.cells] > 0) if fixed is not None else \
            torch.zeros(n, dtype=torch.bool)
        forces = w.get("forces")
        self.Fext = torch.tensor(np.asarray(forces).reshape(-1, 3)[self.cells], dtype=F64) if forces is not None \
            else torch.zeros(n, 3, dtype=F64)
        self.own_signal = w.get("amp") is not None or w.get("phase") is not None
        amp = w.get("amp"); phase = w.get("phase")
        self.amp0 = torch.tensor(np.asarray(amp).reshape(-1)[self.cells] if amp is not None
                                 else np.full(n, p["temp_amp"]), dtype=F64)
        self.phase0 = torch.tensor(np.asarray(phase).reshape(-1)[self.cells] if phase is not None
                                   else np.full(n, p["temp_phase"]), dtype=F64)
        self.dt = self.stable_dt()

    def stable_dt(self):
        """dt = dt_scale / (2 pi max over bonds sqrt(k_b / m_min)) with the
        palette's moduli and densities (Eq. 31-32); without bonds, the
        voxels' own sqrt(E l / m)."""
        l = self.l
        m = self.rho0 * l ** 3
        w2 = []
        for i, j in self.bonds:
            if i.numel():
                Ec = 2 * self.E0[i] * self.E0[j] / (self.E0[i] + self.E0[j])
                w2.append(Ec * l / torch.minimum(m[i], m[j]))
        if w2:
            wmax = math.sqrt(float(torch.cat(w2).max()))
        else:
            wmax = math.sqrt(float((self.E0 * l / m).max())) if self.nvox else 0.0
        dts = self.p.get("dt_scale", 1.0) or 1.0
        return dts / (2 * math.pi * wmax) if wmax > 0 else 0.0


def initial_state(lat, w):
    """(u, q, P, L) at rest, with the workload's initial velocity or state;
    P = m v and L = I w with the palette's masses (the initial velocities
    are what is held fixed)."""
    n = lat.nvox
    u = torch.zeros(n, 3, dtype=F64)
    q = torch.zeros(n, 4, dtype=F64); q[:, 0] = 1.0
    v = torch.zeros(n, 3, dtype=F64)
    om = torch.zeros(n, 3, dtype=F64)
    if w.get("velocity") is not None:
        v = torch.tensor(np.asarray(w["velocity"]).reshape(-1, 3)[lat.cells], dtype=F64)
    st = w.get("state")
    if st is not None:
        u = torch.tensor(st["u"][lat.cells], dtype=F64)
        q = torch.tensor(st["q"][lat.cells], dtype=F64)
        v = torch.tensor(st["v"][lat.cells], dtype=F64)
        om = torch.tensor(st["w"][lat.cells], dtype=F64)
    v = torch.where(lat.fixed.unsqueeze(-1), torch.zeros_like(v), v)
    om = torch.where(lat.fixed.unsqueeze(-1), torch.zeros_like(om), om)
    return u, q, v, om


def rollout(lat, w, steps, E=None, rho=None, phase=None, amp=None):
    """Final (u, q, v, w) per filled voxel after `steps` steps, as functions
    of the per-voxel parameter tensors (None: the palette's / workload's)."""
    p = lat.p
    l, dt = lat.l, lat.dt
    E = lat.E0 if E is None else E
    rho = lat.rho0 if rho is None else rho
    phase = lat.phase0 if phase is None else phase
    amp = lat.amp0 if amp is None else amp
    m = rho * l ** 3
    I = m * l * l / 6.0
    kv = E * l
    cg = 2 * p["zeta_slow"] * torch.sqrt(m * kv)
    cgr = 2 * p["zeta_slow"] * torch.sqrt(I * E * l ** 3 / 6.0)
    cfloor = 2 * p["zeta_col"] * torch.sqrt(m * kv)
    G = E / (2 * (1 + lat.nu))
    consts = []
    for i, j in lat.bonds:
        Ec = 2 * E[i] * E[j] / (E[i] + E[j])
        Gc = 2 * G[i] * G[j] / (G[i] + G[j])
        a1 = Ec * l
        a2 = Gc * l ** 3 / 6.0
        ct = 2 * p["zeta_bond"] * torch.sqrt(torch.minimum(m[i], m[j]) * a1)
        consts.append((a1, a2, ct))
    u, q, v0, om0 = initial_state(lat, w)
    P = m.unsqueeze(-1) * v0
    Lm = I.unsqueeze(-1) * om0
    static = torch.zeros(lat.nvox, dtype=torch.bool)
    g = p["gravity"]
    free = ~lat.fixed
    for n in range(steps):
        t = n * dt
        dT = amp * torch.sin(2 * math.pi * p["temp_freq"] * t + phase)
        eps = lat.cte * dT
        vel = P / m.unsqueeze(-1)
        om = Lm / I.unsqueeze(-1)
        F = torch.zeros_like(u)
        M = torch.zeros_like(u)
        R = _rot_matrix(q)
        for a, ((i, j), (a1, a2, ct)) in enumerate(zip(lat.bonds, consts)):
            if i.numel() == 0:
                continue
            ex, ey, ez = R[i][:, :, a], R[i][:, :, (a + 1) % 3], R[i][:, :, (a + 2) % 3]
            d = u[j] - u[i]
            d = d + torch.nn.functional.one_hot(torch.tensor(a), 3).to(F64) * l
            Lb = l * (1 + 0.5 * (eps[i] + eps[j]))
            X2 = (ex * d).sum(-1) - Lb
            Y2 = (ey * d).sum(-1)
            Z2 = (ez * d).sum(-1)
            th = _log_rotvec(_quat_mul(_quat_conj(q[i]), q[j]))
            tx, ty, tz = th[:, a], th[:, (a + 1) % 3], th[:, (a + 2) % 3]
            b1, b2, b3 = a1, a1 * l / 2, a1 * l * l / 6
            f2 = (a1 * X2, b1 * Y2 - b2 * tz, b1 * Z2 + b2 * ty)
            m2 = (a2 * tx, b2 * Z2 + 2 * b3 * ty, -b2 * Y2 + 2 * b3 * tz)
            m1 = (-a2 * tx, b2 * Z2 + b3 * ty, -b2 * Y2 + b3 * tz)
            back = lambda c: -(c[0].unsqueeze(-1) * ex + c[1].unsqueeze(-1) * ey + c[2].unsqueeze(-1) * ez)
            F2, M2, M1 = back(f2), back(m2), back(m1)
            # bond damping: relative motion without the pair's rigid motion
            wa = 0.5 * (om[i] + om[j])
            Vr = 0.5 * (vel[j] - vel[i]) + torch.cross(0.5 * d, wa, dim=-1)
            wr = 0.5 * (om[j] - om[i])
            cr = ct * l * l / 6
            F2 = F2 - ct.unsqueeze(-1) * Vr
            M2 = M2 - cr.unsqueeze(-1) * wr
            M1 = M1 + cr.unsqueeze(-1) * wr
            F = F.index_add(0, j, F2).index_add(0, i, -F2)
            M = M.index_add(0, j, M2).index_add(0, i, M1)
        F = F + lat.Fext
        F = F - torch.stack([torch.zeros_like(m), torch.zeros_like(m), m * g], -1)
        F = F - cg.unsqueeze(-1) * vel
        M = M - cgr.unsqueeze(-1) * om
        Fn = torch.zeros_like(m)
        if p["floor_on"]:
            pen = 0.5 * l * eps - u[:, 2] - (p["origin"][2] + lat.iz * l)
            Fn = torch.where(pen > 0, torch.clamp(kv * pen - cfloor * vel[:, 2], min=0.0), torch.zeros_like(m))
            F = F + torch.stack([torch.zeros_like(m), torch.zeros_like(m), Fn], -1)
            contact = Fn > 0
            Fl = F[:, :2]
            Fl2 = _sum_sq(Fl)
            Flen = torch.sqrt(torch.where(contact & (Fl2 > 0), Fl2, torch.ones_like(m)))
            Flen = torch.where(contact & (Fl2 > 0), Flen, torch.zeros_like(m))
            Fdiv = torch.where(Flen > 0, Flen, torch.ones_like(m))
            vl = vel[:, :2]
            vlen2 = _sum_sq(vl)
            within_s = Flen <= lat.mu_s * Fn
            hold = contact & static & within_s
            released = contact & static & ~within_s
            moving = contact & ~hold
            halt = moving & (torch.sqrt(vlen2) <= lat.mu_d * Fn * dt / m)
            slide = moving & ~halt
            vlen = torch.sqrt(torch.where(slide, vlen2, torch.ones_like(m)))
            zero2 = torch.zeros_like(Fl)
            Fl_new = torch.where((hold | (halt & within_s)).unsqueeze(-1), zero2, Fl)
            Fl_new = torch.where((halt & ~within_s).unsqueeze(-1),
                                 Fl - (lat.mu_d * Fn / Fdiv).unsqueeze(-1) * Fl, Fl_new)
            Fl_new = torch.where(slide.unsqueeze(-1), Fl - (lat.mu_d * Fn / vlen).unsqueeze(-1) * vl, Fl_new)
            F = torch.cat([Fl_new, F[:, 2:]], -1)
            Pl = torch.where((hold | halt).unsqueeze(-1), torch.zeros_like(Fl), P[:, :2])
            P = torch.cat([Pl, P[:, 2:]], -1)
            static = torch.where(contact, (static & ~released) | halt, torch.zeros_like(static))
            static = static & ~(contact & ~hold & ~halt)
        # integrate (fixed voxels keep u, q and have P = L = 0)
        P_new = P + F * dt
        u_new = u + P_new / m.unsqueeze(-1) * dt
        L_new = Lm + M * dt
        dq = _exp_quat(L_new / I.unsqueeze(-1) * dt)
        q_new = _quat_mul(dq, q)
        q_new = q_new / torch.sqrt(_sum_sq(q_new)).unsqueeze(-1)
        fz = free.unsqueeze(-1)
        P = torch.where(fz, P_new, torch.zeros_like(P))
        Lm = torch.where(fz, L_new, torch.zeros_like(Lm))
        u = torch.where(fz, u_new, u)
        q = torch.where(fz, q_new, q)
    return u, q, P / m.unsqueeze(-1), Lm / I.unsqueeze(-1)


def scatter(lat, a, ncell):
    """Per-voxel rows back to per-cell (zeros at empty cells)."""
    out = np.zeros((ncell,) + tuple(a.shape[1:]))
    out[lat.cells] = a.detach().numpy()
    return out
