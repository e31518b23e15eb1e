// Hand-written reverse-mode derivatives (vector-Jacobian products) of the
// bond force and of the voxel update, for gradients of a trajectory with
// respect to per-voxel stiffness and actuation phase.  Each function
// recomputes the forward intermediates it needs from the same inputs as
// the forward code in vx_device.hpp and walks them backwards; branch
// decisions (series vs library path, floor contact, friction state) are
// those of the forward evaluation.
#pragma once

#include "vx_device.hpp"

namespace vx {

// Adjoint of one voxel's bond inputs: displacement, orientation, velocity,
// angular velocity, thermal strain.
template <typename T>
struct KinAdj {
    T ux, uy, uz, qw, qx, qy, qz, vx, vy, vz, wx, wy, wz, eps;
};

template <typename T>
struct BondAdj {
    KinAdj<T> A, B;
    T a1, a2, ct;   // adjoints of the bond constants
};

// Chain the bond-constant adjoints back to the two voxels' moduli.
template <typename T>
VX_HD void bond_k_from_E_vjp(T EA, T EB, T gA, T gB, const BondK<T> &k, T g_a1, T g_a2, T g_ct,
                             const LatK<T> &C, T *g_EA, T *g_EB) {
    // ct = 2 zeta sqrt(m a1): d ct / d a1 = ct / (2 a1)
    const T ga1 = g_a1 + (k.a1 > T(0) ? g_ct * pdiv(k.ct, T(2) * k.a1) : T(0));
    const T is = pdiv(T(1), EA + EB), is2 = T(2) * is * is;
    const T dEc_dA = EB * EB * is2, dEc_dB = EA * EA * is2;
    const T GA = EA * gA, GB = EB * gB, isg = pdiv(T(1), GA + GB), isg2 = T(2) * isg * isg;
    const T dGc_dA = GB * GB * isg2 * gA, dGc_dB = GA * GA * isg2 * gB;
    const T ga2 = g_a2 * C.l * C.l26;
    *g_EA = ga1 * C.l * dEc_dA + ga2 * dGc_dA;
    *g_EB = ga1 * C.l * dEc_dB + ga2 * dGc_dB;
}

// d/du of atan(sqrt(u))/sqrt(u) on the series range (see atan_over_t).
template <typename T> VX_HD T atan_over_t_d(T u);
template <> VX_HD float atan_over_t_d<float>(float u) {
    float p = 3.0f * (-1.0f / 7.0f);
    p = fmaf(p, u, 2.0f * (1.0f / 5.0f));
    return fmaf(p, u, -1.0f / 3.0f);
}
template <> VX_HD double atan_over_t_d<double>(double u) {
    double p = 7.0 * (-1.0 / 15.0);
    p = fma(p, u, 6.0 * (1.0 / 13.0));
    p = fma(p, u, 5.0 * (-1.0 / 11.0));
    p = fma(p, u, 4.0 * (1.0 / 9.0));
    p = fma(p, u, 3.0 * (-1.0 / 7.0));
    p = fma(p, u, 2.0 * (1.0 / 5.0));
    return fma(p, u, -1.0 / 3.0);
}

// Reverse of bond_core (+ the log map and rotation inputs of bond_eval)
// for a bond along axis AX.  gF, gM1, gM2: adjoints of the bond's outputs
// (force on voxel 2, moments on voxels 1 and 2, world frame).
template <typename T, int AX>
VX_HD BondAdj<T> bond_vjp(const VoxKin<T> &A, const VoxKin<T> &B, const BondK<T> &K, const LatK<T> &C,
                          const T gF[3], const T gM1[3], const T gM2[3]) {
    constexpr int A0 = AX, A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    BondAdj<T> g{};
    // ---- forward recompute ----
    const T du[3] = {B.ux - A.ux, B.uy - A.uy, B.uz - A.uz};
    T d[3] = {du[0], du[1], du[2]};
    d[AX] += C.l;
    const Rot<T> R = rot_of(A.qw, A.qx, A.qy, A.qz);
    const T cv[3][3] = {{R.c[0].x, R.c[0].y, R.c[0].z}, {R.c[1].x, R.c[1].y, R.c[1].z},
                        {R.c[2].x, R.c[2].y, R.c[2].z}};
    const T *ex = cv[A0], *ey = cv[A1], *ez = cv[A2];
    const T rw = A.qw * B.qw + A.qx * B.qx + A.qy * B.qy + A.qz * B.qz;
    const T rx = A.qw * B.qx - A.qx * B.qw - A.qy * B.qz + A.qz * B.qy;
    const T ry = A.qw * B.qy + A.qx * B.qz - A.qy * B.qw - A.qz * B.qx;
    const T rz = A.qw * B.qz - A.qx * B.qy + A.qy * B.qx - A.qz * B.qw;
    const T sg = rw < T(0) ? T(-1) : T(1);
    const T aw = sg * rw;
    const T s2 = rx * rx + ry * ry + rz * rz;
    const T iw = frcp(aw);
    const T u = s2 * iw * iw;
    T k, dk_ds2, dk_daw;
    if (u < Series<T>::kLogU) {
        const T P = atan_over_t(u), Pd = atan_over_t_d(u);
        k = T(2) * iw * P;
        dk_ds2 = T(2) * iw * iw * iw * Pd;
        dk_daw = -T(2) * iw * iw * (P + T(2) * u * Pd);
    } else {
        const T s = dsqrt(s2), n2 = s2 + aw * aw, phi = datan2(s, aw);
        k = T(2) * phi / s;
        const T dk_ds = T(2) * aw / (s * n2) - T(2) * phi / s2;
        dk_ds2 = dk_ds / (T(2) * s);
        dk_daw = -T(2) / n2;
    }
    const T ks = sg * k;
    const T th[3] = {ks * rx, ks * ry, ks * rz};
    const T tx = th[A0], ty = th[A1], tz = th[A2];
    const T eh = T(0.5) * (A.eps + B.eps);
    const T X2 = ex[0] * du[0] + ex[1] * du[1] + ex[2] * du[2] + C.l * (R.dm1[A0] - eh);
    const T Y2 = ey[0] * du[0] + ey[1] * du[1] + ey[2] * du[2] + C.l * ey[AX];
    const T Z2 = ez[0] * du[0] + ez[1] * du[1] + ez[2] * du[2] + C.l * ez[AX];
    const T b1 = K.a1, b2 = K.a1 * C.hl, b3 = K.a1 * C.l26, b3x2 = K.a1 * C.l23;
    const T f2[3] = {K.a1 * X2, b1 * Y2 - b2 * tz, b1 * Z2 + b2 * ty};
    const T m2[3] = {K.a2 * tx, b2 * Z2 + b3x2 * ty, -b2 * Y2 + b3x2 * tz};
    const T m1[3] = {-K.a2 * tx, b2 * Z2 + b3 * ty, -b2 * Y2 + b3 * tz};
    const T h = T(0.5), q4 = T(0.25);
    const T cr = K.ct * C.l26;
    const T ws[3] = {A.wx + B.wx, A.wy + B.wy, A.wz + B.wz};
    const T vr[3] = {h * (B.vx - A.vx) + q4 * (d[1] * ws[2] - d[2] * ws[1]),
                     h * (B.vy - A.vy) + q4 * (d[2] * ws[0] - d[0] * ws[2]),
                     h * (B.vz - A.vz) + q4 * (d[0] * ws[1] - d[1] * ws[0])};
    const T wr[3] = {h * (B.wx - A.wx), h * (B.wy - A.wy), h * (B.wz - A.wz)};

    // ---- reverse ----
    // damping: F2 -= ct vr, M2 -= cr wr, M1 += cr wr
    T g_cr = T(0);
    for (int i = 0; i < 3; ++i) {
        g.ct += -gF[i] * vr[i];
        g_cr += (gM1[i] - gM2[i]) * wr[i];
    }
    g.ct += g_cr * C.l26;
    const T g_vr[3] = {-K.ct * gF[0], -K.ct * gF[1], -K.ct * gF[2]};
    const T g_wr[3] = {cr * (gM1[0] - gM2[0]), cr * (gM1[1] - gM2[1]), cr * (gM1[2] - gM2[2])};
    // vr = (vB - vA)/2 + (d x ws)/4
    T g_d[3], g_ws[3];
    g_d[0] = q4 * (ws[1] * g_vr[2] - ws[2] * g_vr[1]);
    g_d[1] = q4 * (ws[2] * g_vr[0] - ws[0] * g_vr[2]);
    g_d[2] = q4 * (ws[0] * g_vr[1] - ws[1] * g_vr[0]);
    g_ws[0] = q4 * (g_vr[1] * d[2] - g_vr[2] * d[1]);
    g_ws[1] = q4 * (g_vr[2] * d[0] - g_vr[0] * d[2]);
    g_ws[2] = q4 * (g_vr[0] * d[1] - g_vr[1] * d[0]);
    g.B.vx += h * g_vr[0]; g.B.vy += h * g_vr[1]; g.B.vz += h * g_vr[2];
    g.A.vx -= h * g_vr[0]; g.A.vy -= h * g_vr[1]; g.A.vz -= h * g_vr[2];
    g.A.wx += g_ws[0] - h * g_wr[0]; g.A.wy += g_ws[1] - h * g_wr[1]; g.A.wz += g_ws[2] - h * g_wr[2];
    g.B.wx += g_ws[0] + h * g_wr[0]; g.B.wy += g_ws[1] + h * g_wr[1]; g.B.wz += g_ws[2] + h * g_wr[2];
    // back transform: F2 = -(f2x ex + f2y ey + f2z ez), same for M2, M1
    T g_ex[3], g_ey[3], g_ez[3], g_f2[3], g_m2[3], g_m1[3];
    for (int i = 0; i < 3; ++i) {
        g_ex[i] = -(f2[0] * gF[i] + m2[0] * gM2[i] + m1[0] * gM1[i]);
        g_ey[i] = -(f2[1] * gF[i] + m2[1] * gM2[i] + m1[1] * gM1[i]);
        g_ez[i] = -(f2[2] * gF[i] + m2[2] * gM2[i] + m1[2] * gM1[i]);
    }
    g_f2[0] = -(gF[0] * ex[0] + gF[1] * ex[1] + gF[2] * ex[2]);
    g_f2[1] = -(gF[0] * ey[0] + gF[1] * ey[1] + gF[2] * ey[2]);
    g_f2[2] = -(gF[0] * ez[0] + gF[1] * ez[1] + gF[2] * ez[2]);
    g_m2[0] = -(gM2[0] * ex[0] + gM2[1] * ex[1] + gM2[2] * ex[2]);
    g_m2[1] = -(gM2[0] * ey[0] + gM2[1] * ey[1] + gM2[2] * ey[2]);
    g_m2[2] = -(gM2[0] * ez[0] + gM2[1] * ez[1] + gM2[2] * ez[2]);
    g_m1[0] = -(gM1[0] * ex[0] + gM1[1] * ex[1] + gM1[2] * ex[2]);
    g_m1[1] = -(gM1[0] * ey[0] + gM1[1] * ey[1] + gM1[2] * ey[2]);
    g_m1[2] = -(gM1[0] * ez[0] + gM1[1] * ez[1] + gM1[2] * ez[2]);
    // local forces
    T g_X2 = g_f2[0] * K.a1;
    T g_Y2 = g_f2[1] * b1 - g_m2[2] * b2 - g_m1[2] * b2;
    T g_Z2 = g_f2[2] * b1 + g_m2[1] * b2 + g_m1[1] * b2;
    T g_tx = g_m2[0] * K.a2 - g_m1[0] * K.a2;
    T g_ty = g_f2[2] * b2 + g_m2[1] * b3x2 + g_m1[1] * b3;
    T g_tz = -g_f2[1] * b2 + g_m2[2] * b3x2 + g_m1[2] * b3;
    g.a1 += g_f2[0] * X2;
    g.a2 += g_m2[0] * tx - g_m1[0] * tx;
    const T g_b1 = g_f2[1] * Y2 + g_f2[2] * Z2;
    const T g_b2 = -g_f2[1] * tz + g_f2[2] * ty + g_m2[1] * Z2 - g_m2[2] * Y2 + g_m1[1] * Z2 - g_m1[2] * Y2;
    const T g_b3 = g_m1[1] * ty + g_m1[2] * tz;
    const T g_b3x2 = g_m2[1] * ty + g_m2[2] * tz;
    g.a1 += g_b1 + g_b2 * C.hl + g_b3 * C.l26 + g_b3x2 * C.l23;
    // X2, Y2, Z2
    T g_du[3], g_dm1a = g_X2 * C.l;
    for (int i = 0; i < 3; ++i) {
        g_ex[i] += g_X2 * du[i];
        g_ey[i] += g_Y2 * du[i];
        g_ez[i] += g_Z2 * du[i];
        g_du[i] = g_X2 * ex[i] + g_Y2 * ey[i] + g_Z2 * ez[i] + g_d[i];
    }
    g_ey[AX] += g_Y2 * C.l;
    g_ez[AX] += g_Z2 * C.l;
    g.A.eps -= h * g_X2 * C.l;
    g.B.eps -= h * g_X2 * C.l;
    // displacements
    g.B.ux += g_du[0]; g.B.uy += g_du[1]; g.B.uz += g_du[2];
    g.A.ux -= g_du[0]; g.A.uy -= g_du[1]; g.A.uz -= g_du[2];
    // log map: th = ks (rx, ry, rz)
    T g_th[3];
    g_th[A0] = g_tx; g_th[A1] = g_ty; g_th[A2] = g_tz;
    const T g_ks = g_th[0] * rx + g_th[1] * ry + g_th[2] * rz;
    const T g_k = sg * g_ks;
    const T g_s2 = g_k * dk_ds2, g_aw = g_k * dk_daw;
    const T g_rx = ks * g_th[0] + T(2) * g_s2 * rx;
    const T g_ry = ks * g_th[1] + T(2) * g_s2 * ry;
    const T g_rz = ks * g_th[2] + T(2) * g_s2 * rz;
    const T g_rw = sg * g_aw;
    // r = conj(qA) (x) qB
    g.A.qw += g_rw * B.qw + g_rx * B.qx + g_ry * B.qy + g_rz * B.qz;
    g.A.qx += g_rw * B.qx - g_rx * B.qw + g_ry * B.qz - g_rz * B.qy;
    g.A.qy += g_rw * B.qy - g_rx * B.qz - g_ry * B.qw + g_rz * B.qx;
    g.A.qz += g_rw * B.qz + g_rx * B.qy - g_ry * B.qx - g_rz * B.qw;
    g.B.qw += g_rw * A.qw - g_rx * A.qx - g_ry * A.qy - g_rz * A.qz;
    g.B.qx += g_rw * A.qx + g_rx * A.qw - g_ry * A.qz + g_rz * A.qy;
    g.B.qy += g_rw * A.qy + g_rx * A.qz + g_ry * A.qw - g_rz * A.qx;
    g.B.qz += g_rw * A.qz - g_rx * A.qy + g_ry * A.qx + g_rz * A.qw;
    // rotation matrix of qA: gradients of its columns and diagonal terms
    T gc[3][3];
    for (int i = 0; i < 3; ++i) { gc[A0][i] = g_ex[i]; gc[A1][i] = g_ey[i]; gc[A2][i] = g_ez[i]; }
    T gdm1[3] = {gc[0][0], gc[1][1], gc[2][2]};   // c_i[i] = 1 + dm1[i]
    gdm1[A0] += g_dm1a;
    const T w = A.qw, x = A.qx, y = A.qy, z = A.qz;
    T gw = T(0), gx = T(0), gy = T(0), gz = T(0);
    // dm1 = (-2(y^2+z^2), -2(x^2+z^2), -2(x^2+y^2))
    gx += -T(4) * x * (gdm1[1] + gdm1[2]);
    gy += -T(4) * y * (gdm1[0] + gdm1[2]);
    gz += -T(4) * z * (gdm1[0] + gdm1[1]);
    // off-diagonals
    const T c0y = gc[0][1], c0z = gc[0][2], c1x = gc[1][0], c1z = gc[1][2], c2x = gc[2][0], c2y = gc[2][1];
    // c0.y = 2(xy + wz), c1.x = 2(xy - wz)
    gx += T(2) * y * (c0y + c1x); gy += T(2) * x * (c0y + c1x);
    gw += T(2) * z * (c0y - c1x); gz += T(2) * w * (c0y - c1x);
    // c0.z = 2(xz - wy), c2.x = 2(xz + wy)
    gx += T(2) * z * (c0z + c2x); gz += T(2) * x * (c0z + c2x);
    gw += T(2) * y * (c2x - c0z); gy += T(2) * w * (c2x - c0z);
    // c1.z = 2(yz + wx), c2.y = 2(yz - wx)
    gy += T(2) * z * (c1z + c2y); gz += T(2) * y * (c1z + c2y);
    gw += T(2) * x * (c1z - c2y); gx += T(2) * w * (c1z - c2y);
    g.A.qw += gw; g.A.qx += gx; g.A.qy += gy; g.A.qz += gz;
    return g;
}

// Adjoint of update_core.
template <typename T>
struct UpdAdj {
    VoxRaw<T> r;         // state at t_n
    T Fx, Fy, Fz, Mx, My, Mz;   // bond sums
    T eps;
    T kv, cg, cgr, cfloor;      // per-voxel constants
    T m, inv_m, inv_I;          // mass terms (each taken as an independent input)
};

// d cos(h)/da2 and d (sin(h)/(2h))/da2 with a2 = (2h)^2, on the series range.
template <typename T>
VX_HD void half_angle_series_d(T a2, T *dc, T *dsk) {
    const T h2 = T(0.25) * a2;
    if constexpr (sizeof(T) == 8) {
        double pc = 4.0 / 40320.0;
        pc = fma(pc, h2, -3.0 / 720.0);
        pc = fma(pc, h2, 2.0 / 24.0);
        pc = fma(pc, h2, -0.5);
        *dc = T(0.25) * pc;
        double ps = 4.0 / 362880.0;
        ps = fma(ps, h2, -3.0 / 5040.0);
        ps = fma(ps, h2, 2.0 / 120.0);
        ps = fma(ps, h2, -1.0 / 6.0);
        *dsk = T(0.125) * ps;
    } else {
        float pc = 2.0f / 24.0f;
        pc = fmaf(pc, h2, -0.5f);
        *dc = 0.25f * pc;
        float ps = 2.0f / 120.0f;
        ps = fmaf(ps, h2, -1.0f / 6.0f);
        *dsk = 0.125f * ps;
    }
}

// Reverse of update_core: g is the adjoint of the state at t_n+1; returns
// the adjoints of its inputs.  The friction state and branch are those of
// the forward evaluation with the same inputs.
template <typename T>
VX_HD UpdAdj<T> update_vjp(const UpdEnv<T> &e, uint8_t fl, const MatConst<T> &mc, T eps, const VoxRaw<T> &r,
                           T Fx, T Fy, T Fz, T Mx, T My, T Mz, const VoxRaw<T> &g) {
    UpdAdj<T> a{};
    if (fl & FLAG_FIXED) {
        a.r.ux = g.ux; a.r.uy = g.uy; a.r.uz = g.uz;
        a.r.qw = g.qw; a.r.qx = g.qx; a.r.qy = g.qy; a.r.qz = g.qz;
        return a;
    }
    // ---- forward recompute ----
    T px = r.px, py = r.py, pz = r.pz;
    if (fl & FLAG_FORCED) { Fx += e.Fext[0]; Fy += e.Fext[1]; Fz += e.Fext[2]; }
    Fz -= mc.m * e.gravity;
    const T vx = px * mc.inv_m, vy = py * mc.inv_m, vz = pz * mc.inv_m;
    const T wx = r.lx * mc.inv_I, wy = r.ly * mc.inv_I, wz = r.lz * mc.inv_I;
    Fx -= vx * mc.cg; Fy -= vy * mc.cg; Fz -= vz * mc.cg;
    Mx -= wx * mc.cgr; My -= wy * mc.cgr; Mz -= wz * mc.cgr;
    T Fn = T(0), pen = T(0);
    bool contact = false;
    if (e.floor_on) {
        pen = T(0.5) * e.l * eps - r.uz - e.z0;
        if (pen > T(0)) {
            Fn = mc.kv * pen - mc.cfloor * vz;
            contact = Fn > T(0);
            if (!contact) Fn = T(0);
            Fz += Fn;
        }
    }
    if (fl & FLAG_CAND) { Fx += e.Fc[0]; Fy += e.Fc[1]; Fz += e.Fc[2]; }
    const T Flx = Fx, Fly = Fy;               // lateral force before friction
    int branch = FR_NONE;
    T Fl = T(0), vl = T(0);
    if (e.floor_on && Fn > T(0)) {
        Fl = dsqrt(Fx * Fx + Fy * Fy);
        bool done = false;
        if (fl & FLAG_STATIC) {
            if (Fl <= mc.mu_s * Fn) { Fx = Fy = T(0); px = py = T(0); done = true; branch = FR_HOLD; }
        }
        if (!done) {
            vl = dsqrt(vx * vx + vy * vy);
            if (vl <= mc.mu_d * Fn * e.dt * mc.inv_m) {
                px = py = T(0);
                if (Fl <= mc.mu_s * Fn) { Fx = Fy = T(0); branch = FR_HALT_HOLD; }
                else { const T f = mc.mu_d * Fn / Fl; Fx -= f * Fx; Fy -= f * Fy; branch = FR_HALT_SLIDE; }
            } else {
                const T f = mc.mu_d * Fn / vl;
                Fx -= f * vx; Fy -= f * vy;
                branch = FR_SLIDE;
            }
        }
    }
    const T dt = e.dt;
    const T Px = px + Fx * dt, Py = py + Fy * dt, Pz = pz + Fz * dt;
    const T Lx = r.lx + Mx * dt, Ly = r.ly + My * dt, Lz = r.lz + Mz * dt;
    const T rx = Lx * mc.inv_I * dt, ry = Ly * mc.inv_I * dt, rz = Lz * mc.inv_I * dt;
    const T a2 = rx * rx + ry * ry + rz * rz;
    T dw, sk, ddw, dsk;
    if (a2 < Series<T>::kExpA2) {
        half_angle_series(a2, &dw, &sk);
        half_angle_series_d(a2, &ddw, &dsk);
    } else {
        const T ang = dsqrt(a2), hh = T(0.5) * ang;
        T sn, cs;
        dsincos(hh, &sn, &cs);
        dw = cs;
        sk = sn / ang;
        ddw = -sk * T(0.25);
        dsk = (hh * cs - sn) / (T(16) * hh * hh * hh);
    }
    const T dx = sk * rx, dy = sk * ry, dz = sk * rz;
    const T qw = r.qw, qx = r.qx, qy = r.qy, qz = r.qz;
    const T nw = dw * qw - dx * qx - dy * qy - dz * qz;
    const T nx = dw * qx + dx * qw + dy * qz - dz * qy;
    const T ny = dw * qy - dx * qz + dy * qw + dz * qx;
    const T nz = dw * qz + dx * qy - dy * qx + dz * qw;
    const T n2 = nw * nw + nx * nx + ny * ny + nz * nz;
    const T dn = n2 - T(1);
    T inv, dinv;
    if (dn < Series<T>::kNormD && dn > -Series<T>::kNormD) {
        inv = fma(dn, fma(dn, T(0.375), T(-0.5)), T(1));
        dinv = fma(dn, T(0.75), T(-0.5));
    } else {
        const T s = dsqrt(n2);
        inv = T(1) / s;
        dinv = -T(0.5) * inv / n2;
    }
    // ---- reverse ----
    // q' = (nw, nx, ny, nz) inv(n2)
    const T gdot = g.qw * nw + g.qx * nx + g.qy * ny + g.qz * nz;
    const T t2 = T(2) * gdot * dinv;
    const T gnw = inv * g.qw + t2 * nw, gnx = inv * g.qx + t2 * nx;
    const T gny = inv * g.qy + t2 * ny, gnz = inv * g.qz + t2 * nz;
    // n = dq (x) q: g_dq = g_n (x) conj(q), g_q = conj(dq) (x) g_n
    const T gdw = gnw * qw + gnx * qx + gny * qy + gnz * qz;
    const T gdx = -gnw * qx + gnx * qw - gny * qz + gnz * qy;
    const T gdy = -gnw * qy + gnx * qz + gny * qw - gnz * qx;
    const T gdz = -gnw * qz - gnx * qy + gny * qx + gnz * qw;
    a.r.qw = dw * gnw + dx * gnx + dy * gny + dz * gnz;
    a.r.qx = dw * gnx - dx * gnw - dy * gnz + dz * gny;
    a.r.qy = dw * gny + dx * gnz - dy * gnw - dz * gnx;
    a.r.qz = dw * gnz - dx * gny + dy * gnx - dz * gnw;
    // dq = (dw, sk r)
    const T gsk = gdx * rx + gdy * ry + gdz * rz;
    const T ga2 = gdw * ddw + gsk * dsk;
    const T grx = sk * gdx + T(2) * ga2 * rx, gry = sk * gdy + T(2) * ga2 * ry, grz = sk * gdz + T(2) * ga2 * rz;
    // r = L' inv_I dt; L' = L + M dt
    const T c = mc.inv_I * dt;
    a.inv_I += (grx * Lx + gry * Ly + grz * Lz) * dt;
    const T gLx = g.lx + grx * c, gLy = g.ly + gry * c, gLz = g.lz + grz * c;
    a.r.lx = gLx; a.r.ly = gLy; a.r.lz = gLz;
    T gMx = gLx * dt, gMy = gLy * dt, gMz = gLz * dt;
    // u' = u + P' inv_m dt; P' = P + F dt
    a.r.ux = g.ux; a.r.uy = g.uy; a.r.uz = g.uz;
    a.inv_m += (g.ux * Px + g.uy * Py + g.uz * Pz) * dt;
    const T gPx = g.px + g.ux * dt * mc.inv_m, gPy = g.py + g.uy * dt * mc.inv_m, gPz = g.pz + g.uz * dt * mc.inv_m;
    T gFx = gPx * dt, gFy = gPy * dt, gFz = gPz * dt;     // adjoint of F after friction
    T gpx = gPx, gpy = gPy, gpz = gPz;                    // adjoint of P after friction
    T gvx = T(0), gvy = T(0), gvz = T(0), gFn = T(0);
    // friction (lateral components)
    if (branch == FR_HOLD || branch == FR_HALT_HOLD) {
        gFx = gFy = T(0);
        gpx = gpy = T(0);
    } else if (branch == FR_HALT_SLIDE) {
        gpx = gpy = T(0);
        const T cc = mc.mu_d * Fn;
        const T dotg = Flx * gFx + Fly * gFy;
        const T k1 = T(1) - cc / Fl, k2 = cc * dotg / (Fl * Fl * Fl);
        const T gcc = -(Flx * gFx + Fly * gFy) / Fl;
        gFx = k1 * gFx + k2 * Flx;
        gFy = k1 * gFy + k2 * Fly;
        gFn += mc.mu_d * gcc;
    } else if (branch == FR_SLIDE) {
        const T cc = mc.mu_d * Fn;
        const T dotv = vx * gFx + vy * gFy;
        gvx += -cc * (gFx / vl - dotv * vx / (vl * vl * vl));
        gvy += -cc * (gFy / vl - dotv * vy / (vl * vl * vl));
        gFn += mc.mu_d * (-dotv / vl);
    }
    // floor normal force
    T guz = T(0);
    if (contact) {
        gFn += gFz;
        a.kv += gFn * pen;
        a.cfloor += -gFn * vz;
        gvz += -gFn * mc.cfloor;
        const T gpen = gFn * mc.kv;
        a.eps += T(0.5) * e.l * gpen;
        guz -= gpen;
    }
    a.r.uz += guz;
    // ground damping
    a.cg += -(gFx * vx + gFy * vy + gFz * vz);
    gvx += -mc.cg * gFx; gvy += -mc.cg * gFy; gvz += -mc.cg * gFz;
    a.cgr += -(gMx * wx + gMy * wy + gMz * wz);
    const T gwx = -mc.cgr * gMx, gwy = -mc.cgr * gMy, gwz = -mc.cgr * gMz;
    a.Fx = gFx; a.Fy = gFy; a.Fz = gFz;
    a.Mx = gMx; a.My = gMy; a.Mz = gMz;
    // gravity (Fz -= m g), and v = P inv_m, w = L inv_I at t_n
    a.m += -e.gravity * gFz;
    a.inv_m += gvx * r.px + gvy * r.py + gvz * r.pz;
    a.inv_I += gwx * r.lx + gwy * r.ly + gwz * r.lz;
    a.r.px = gpx + mc.inv_m * gvx; a.r.py = gpy + mc.inv_m * gvy; a.r.pz = gpz + mc.inv_m * gvz;
    a.r.lx += mc.inv_I * gwx; a.r.ly += mc.inv_I * gwy; a.r.lz += mc.inv_I * gwz;
    return a;
}

}  // namespace vx
