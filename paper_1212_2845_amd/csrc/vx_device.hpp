// Device-side physics of one bond and one voxel update, templated on the
// state precision.  Used by every step kernel (split and fused), so all
// paths compute bit-identical per-bond and per-voxel results.
#pragma once

#include "vx_types.hpp"

namespace vx {

template <typename T> struct V3 { T x, y, z; };

template <typename T> __device__ __forceinline__ T dsqrt(T a);
template <> __device__ __forceinline__ float dsqrt<float>(float a) { return sqrtf(a); }
template <> __device__ __forceinline__ double dsqrt<double>(double a) { return sqrt(a); }
template <typename T> __device__ __forceinline__ T datan2(T y, T x);
template <> __device__ __forceinline__ float datan2<float>(float y, float x) { return atan2f(y, x); }
template <> __device__ __forceinline__ double datan2<double>(double y, double x) { return atan2(y, x); }
template <typename T> __device__ __forceinline__ void dsincos(T a, T *s, T *c);
template <> __device__ __forceinline__ void dsincos<float>(float a, float *s, float *c) { sincosf(a, s, c); }
template <> __device__ __forceinline__ void dsincos<double>(double a, double *s, double *c) { sincos(a, s, c); }
template <typename T> __device__ __forceinline__ bool dfinite(T a);
template <> __device__ __forceinline__ bool dfinite<float>(float a) { return isfinite(a); }
template <> __device__ __forceinline__ bool dfinite<double>(double a) { return isfinite(a); }

// Kinematic quantities of one voxel that its bonds read.
template <typename T>
struct VoxKin {
    T ux, uy, uz;          // displacement from rest
    T qw, qx, qy, qz;      // orientation (body -> world)
    T vx, vy, vz;          // velocity P / m
    T wx, wy, wz;          // angular velocity phi / I
    T eps;                 // thermal strain at t_n
};

// Columns of the rotation matrix of a unit quaternion (body -> world).
template <typename T>
struct Rot {
    V3<T> c[3];
};

template <typename T>
__device__ __forceinline__ Rot<T> rot_of(T w, T x, T y, T z) {
    Rot<T> R;
    const T one = T(1), two = T(2);
    R.c[0] = {one - two * (y * y + z * z), two * (x * y + w * z), two * (x * z - w * y)};
    R.c[1] = {two * (x * y - w * z), one - two * (x * x + z * z), two * (y * z + w * x)};
    R.c[2] = {two * (x * z + w * y), two * (y * z - w * x), one - two * (x * x + y * y)};
    return R;
}

// Result of one bond: force on voxel 2 (voxel 1 gets its negative) and the
// moments on voxel 1 and voxel 2, all in the world frame.
template <typename T>
struct BondOut {
    T f2x, f2y, f2z;
    T m1x, m1y, m1z;
    T m2x, m2y, m2z;
};

// One beam bond along lattice axis AX between voxel A (lower index, voxel
// 1) and voxel B (voxel 2).  Co-rotational: the bond is expressed in the
// frame of voxel 1 with the axis permuted onto +x, where only voxel 2's six
// displacements remain (reduced forces of Eq. 13-24, with the z-force sign
// of the full matrix Eq. 7); the result is rotated back to the world frame
// and bond damping (Eq. 33-35) is added.
template <typename T, int AX>
__device__ __forceinline__ BondOut<T> bond_eval(const VoxKin<T> &A, const Rot<T> &RA,
                                                const VoxKin<T> &B, const PairConst<T> &pc, T l) {
    constexpr int A0 = AX, A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    // world separation of the two centres
    T d[3] = {B.ux - A.ux, B.uy - A.uy, B.uz - A.uz};
    d[AX] += l;
    const V3<T> ex = RA.c[A0], ey = RA.c[A1], ez = RA.c[A2];
    const T dlx = ex.x * d[0] + ex.y * d[1] + ex.z * d[2];
    const T dly = ey.x * d[0] + ey.y * d[1] + ey.z * d[2];
    const T dlz = ez.x * d[0] + ez.y * d[1] + ez.z * d[2];
    // relative rotation q_A^-1 q_B as a rotation vector in A's body frame
    T rw = A.qw * B.qw + A.qx * B.qx + A.qy * B.qy + A.qz * B.qz;
    T rx = A.qw * B.qx - A.qx * B.qw - A.qy * B.qz + A.qz * B.qy;
    T ry = A.qw * B.qy + A.qx * B.qz - A.qy * B.qw - A.qz * B.qx;
    T rz = A.qw * B.qz - A.qx * B.qy + A.qy * B.qx - A.qz * B.qw;
    if (rw < T(0)) { rw = -rw; rx = -rx; ry = -ry; rz = -rz; }
    const T s = dsqrt(rx * rx + ry * ry + rz * rz);
    const T k = (s > T(0)) ? T(2) * datan2(s, rw) / s : T(2) / rw;
    const T th[3] = {k * rx, k * ry, k * rz};
    const T tx = th[A0], ty = th[A1], tz = th[A2];
    // rest length stretched by the mean thermal strain (Eq. 40)
    const T L = l * (T(1) + T(0.5) * (A.eps + B.eps));
    const T X2 = dlx - L, Y2 = dly, Z2 = dlz;
    // local nodal forces K u (u1 = 0)
    const T f2x = pc.a1 * X2;
    const T f2y = pc.b1 * Y2 - pc.b2 * tz;
    const T f2z = pc.b1 * Z2 + pc.b2 * ty;
    const T m2x = pc.a2 * tx;
    const T m2y = pc.b2 * Z2 + T(2) * pc.b3 * ty;
    const T m2z = -pc.b2 * Y2 + T(2) * pc.b3 * tz;
    const T m1x = -m2x;
    const T m1y = pc.b2 * Z2 + pc.b3 * ty;
    const T m1z = -pc.b2 * Y2 + pc.b3 * tz;
    BondOut<T> o;
    // the bond acts with the opposite of K u, rotated back to the world
    o.f2x = -(f2x * ex.x + f2y * ey.x + f2z * ez.x);
    o.f2y = -(f2x * ex.y + f2y * ey.y + f2z * ez.y);
    o.f2z = -(f2x * ex.z + f2y * ey.z + f2z * ez.z);
    o.m2x = -(m2x * ex.x + m2y * ey.x + m2z * ez.x);
    o.m2y = -(m2x * ex.y + m2y * ey.y + m2z * ez.y);
    o.m2z = -(m2x * ex.z + m2y * ey.z + m2z * ez.z);
    o.m1x = -(m1x * ex.x + m1y * ey.x + m1z * ez.x);
    o.m1y = -(m1x * ex.y + m1y * ey.y + m1z * ez.y);
    o.m1z = -(m1x * ex.z + m1y * ey.z + m1z * ez.z);
    // bond damping: relative velocity without the pair's rigid motion
    const T h = T(0.5), q4 = T(0.25);
    const T wax = A.wx + B.wx, way = A.wy + B.wy, waz = A.wz + B.wz;
    const T vrx = h * (B.vx - A.vx) + q4 * (d[1] * waz - d[2] * way);
    const T vry = h * (B.vy - A.vy) + q4 * (d[2] * wax - d[0] * waz);
    const T vrz = h * (B.vz - A.vz) + q4 * (d[0] * way - d[1] * wax);
    const T wrx = h * (B.wx - A.wx), wry = h * (B.wy - A.wy), wrz = h * (B.wz - A.wz);
    o.f2x -= pc.ct * vrx; o.f2y -= pc.ct * vry; o.f2z -= pc.ct * vrz;
    o.m2x -= pc.cr * wrx; o.m2y -= pc.cr * wry; o.m2z -= pc.cr * wrz;
    o.m1x += pc.cr * wrx; o.m1y += pc.cr * wry; o.m1z += pc.cr * wrz;
    return o;
}

// Thermal strain of a voxel at t_n: cte times its temperature signal.
template <typename T>
__device__ __forceinline__ T voxel_strain(const StepArgs<T> &a, long long c, uint8_t fl, T cte) {
    T dT = a.dT_global;
    if (fl & FLAG_ACT) {
        const double arg = a.wt + (double)a.act_phase[c];
        dT = a.act_amp[c] * (T)sin(arg);
    }
    return cte * dT;
}

template <typename T>
__device__ __forceinline__ VoxKin<T> load_kin(const T *__restrict__ s, long long stride, long long c,
                                              const MatConst<T> &mc, T eps) {
    VoxKin<T> k;
    k.ux = s[W_UX * stride + c]; k.uy = s[W_UY * stride + c]; k.uz = s[W_UZ * stride + c];
    k.qw = s[W_QW * stride + c]; k.qx = s[W_QX * stride + c];
    k.qy = s[W_QY * stride + c]; k.qz = s[W_QZ * stride + c];
    k.vx = s[W_PX * stride + c] * mc.inv_m; k.vy = s[W_PY * stride + c] * mc.inv_m;
    k.vz = s[W_PZ * stride + c] * mc.inv_m;
    k.wx = s[W_LX * stride + c] * mc.inv_I; k.wy = s[W_LY * stride + c] * mc.inv_I;
    k.wz = s[W_LZ * stride + c] * mc.inv_I;
    k.eps = eps;
    return k;
}

// Everything after the bond sum for one voxel: external force, gravity,
// ground damping, floor, contact, Coulomb friction, then the synchronous
// "double Euler" update (Eq. 27-30) with the orientation advanced by the
// exact rotation w dt.  Writes the new state of cell c.
template <typename T>
__device__ __forceinline__ void voxel_update(const StepArgs<T> &a, long long c, uint8_t fl,
                                             const MatConst<T> &mc, T eps, T Fx, T Fy, T Fz,
                                             T Mx, T My, T Mz, T *vmax_local) {
    const T *__restrict__ s = a.s_in;
    T *__restrict__ o = a.s_out;
    const long long st = a.stride;
    T ux = s[W_UX * st + c], uy = s[W_UY * st + c], uz = s[W_UZ * st + c];
    T qw = s[W_QW * st + c], qx = s[W_QX * st + c], qy = s[W_QY * st + c], qz = s[W_QZ * st + c];
    T px = s[W_PX * st + c], py = s[W_PY * st + c], pz = s[W_PZ * st + c];
    T lx = s[W_LX * st + c], ly = s[W_LY * st + c], lz = s[W_LZ * st + c];
    if (fl & FLAG_FIXED) {
        o[W_UX * st + c] = ux; o[W_UY * st + c] = uy; o[W_UZ * st + c] = uz;
        o[W_QW * st + c] = qw; o[W_QX * st + c] = qx; o[W_QY * st + c] = qy; o[W_QZ * st + c] = qz;
        o[W_PX * st + c] = T(0); o[W_PY * st + c] = T(0); o[W_PZ * st + c] = T(0);
        o[W_LX * st + c] = T(0); o[W_LY * st + c] = T(0); o[W_LZ * st + c] = T(0);
        return;
    }
    if (fl & FLAG_FORCED) {
        int lo = 0, hi = a.n_forced - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((long long)a.forced_cells[mid] < c) lo = mid + 1; else hi = mid;
        }
        Fx += a.forced_F[3 * lo]; Fy += a.forced_F[3 * lo + 1]; Fz += a.forced_F[3 * lo + 2];
    }
    Fz -= mc.m * a.gravity;
    const T vx = px * mc.inv_m, vy = py * mc.inv_m, vz = pz * mc.inv_m;
    const T wx = lx * mc.inv_I, wy = ly * mc.inv_I, wz = lz * mc.inv_I;
    Fx -= vx * mc.cg; Fy -= vy * mc.cg; Fz -= vz * mc.cg;
    Mx -= wx * mc.cgr; My -= wy * mc.cgr; Mz -= wz * mc.cgr;
    T Fn = T(0);
    if (a.floor_on) {
        const long long nxy = (long long)a.nx * a.ny;
        const int iz = (int)(c / nxy);
        const T Dz = a.origin_z + (T(iz) + T(0.5)) * a.l + uz;
        const T pen = T(0.5) * a.l * (T(1) + eps) - Dz;
        if (pen > T(0)) {
            Fn = mc.kv * pen - mc.cfloor * vz;
            if (Fn < T(0)) Fn = T(0);
            Fz += Fn;
        }
    }
    if (fl & FLAG_CAND) {
        Fx += a.contact_F[c]; Fy += a.contact_F[st + c]; Fz += a.contact_F[2 * st + c];
    }
    // Coulomb friction against the floor (Eq. 36-38)
    uint8_t nf = fl;
    if (a.floor_on) {
        if (Fn > T(0)) {
            const T Fl = dsqrt(Fx * Fx + Fy * Fy);
            bool done = false;
            if (nf & FLAG_STATIC) {
                if (Fl <= mc.mu_s * Fn) {
                    Fx = T(0); Fy = T(0); px = T(0); py = T(0);
                    done = true;
                } else {
                    nf &= (uint8_t)~FLAG_STATIC;
                }
            }
            if (!done) {
                const T vl = dsqrt(vx * vx + vy * vy);
                if (vl <= mc.mu_d * Fn * a.dt * mc.inv_m) {
                    px = T(0); py = T(0);
                    nf |= FLAG_STATIC;
                    if (Fl <= mc.mu_s * Fn) {
                        Fx = T(0); Fy = T(0);
                    } else {
                        const T f = mc.mu_d * Fn / Fl;
                        Fx -= f * Fx; Fy -= f * Fy;
                    }
                } else {
                    const T f = mc.mu_d * Fn / vl;
                    Fx -= f * vx; Fy -= f * vy;
                }
            }
        } else {
            nf &= (uint8_t)~FLAG_STATIC;
        }
        if (nf != fl) a.flags[c] = nf;
    }
    // integrate
    const T dt = a.dt;
    px += Fx * dt; py += Fy * dt; pz += Fz * dt;
    const T nvx = px * mc.inv_m, nvy = py * mc.inv_m, nvz = pz * mc.inv_m;
    ux += nvx * dt; uy += nvy * dt; uz += nvz * dt;
    lx += Mx * dt; ly += My * dt; lz += Mz * dt;
    const T rx = lx * mc.inv_I * dt, ry = ly * mc.inv_I * dt, rz = lz * mc.inv_I * dt;
    const T ang = dsqrt(rx * rx + ry * ry + rz * rz);
    T dw = T(1), sk = T(0.5);
    if (ang > T(0)) {
        T sn, cs;
        dsincos(T(0.5) * ang, &sn, &cs);
        dw = cs;
        sk = sn / ang;
    }
    const T dx = sk * rx, dy = sk * ry, dz = sk * rz;
    // dq * q, then normalise
    T nw = dw * qw - dx * qx - dy * qy - dz * qz;
    T nx = dw * qx + dx * qw + dy * qz - dz * qy;
    T ny = dw * qy - dx * qz + dy * qw + dz * qx;
    T nz = dw * qz + dx * qy - dy * qx + dz * qw;
    const T qn = dsqrt(nw * nw + nx * nx + ny * ny + nz * nz);
    nw /= qn; nx /= qn; ny /= qn; nz /= qn;
    o[W_UX * st + c] = ux; o[W_UY * st + c] = uy; o[W_UZ * st + c] = uz;
    o[W_QW * st + c] = nw; o[W_QX * st + c] = nx; o[W_QY * st + c] = ny; o[W_QZ * st + c] = nz;
    o[W_PX * st + c] = px; o[W_PY * st + c] = py; o[W_PZ * st + c] = pz;
    o[W_LX * st + c] = lx; o[W_LY * st + c] = ly; o[W_LZ * st + c] = lz;
    const bool ok = dfinite(ux) && dfinite(uy) && dfinite(uz) && dfinite(nw) && dfinite(nx) &&
                    dfinite(ny) && dfinite(nz) && dfinite(px) && dfinite(py) && dfinite(pz) &&
                    dfinite(lx) && dfinite(ly) && dfinite(lz);
    if (!ok) atomicOr(a.err_flag, 1u);
    const T sp = dsqrt(nvx * nvx + nvy * nvy + nvz * nvz);
    if (sp > *vmax_local) *vmax_local = sp;
}

}  // namespace vx
