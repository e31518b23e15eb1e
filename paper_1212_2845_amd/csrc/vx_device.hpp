// Device-side physics of one bond and one voxel update, templated on the
// state precision.  Used by every step kernel (split and fused).  Each
// kernel inlines its own copies, which the compiler may contract into FMAs
// differently, so the paths agree to rounding rather than bitwise.
#pragma once

#include "vx_types.hpp"

// The per-bond and per-voxel math compiles for the host too (for unit
// checks of the hand-written derivatives); kernels use it on the device.
#define VX_HD __host__ __device__ __forceinline__

namespace vx {

template <typename T> struct V3 { T x, y, z; };

template <int I, typename T>
VX_HD T comp(const V3<T> &v) {
    if constexpr (I == 0) return v.x;
    else if constexpr (I == 1) return v.y;
    else return v.z;
}

template <typename T> VX_HD T dsqrt(T a);
template <> VX_HD float dsqrt<float>(float a) { return sqrtf(a); }
template <> VX_HD double dsqrt<double>(double a) { return sqrt(a); }
template <typename T> VX_HD T datan2(T y, T x);
template <> VX_HD float datan2<float>(float y, float x) { return atan2f(y, x); }
template <> VX_HD double datan2<double>(double y, double x) { return atan2(y, x); }
template <typename T> VX_HD void dsincos(T a, T *s, T *c);
template <> VX_HD void dsincos<float>(float a, float *s, float *c) { sincosf(a, s, c); }
template <> VX_HD void dsincos<double>(double a, double *s, double *c) { sincos(a, s, c); }
template <typename T> VX_HD bool dfinite(T a);
template <> VX_HD bool dfinite<float>(float a) { return isfinite(a); }
template <> VX_HD bool dfinite<double>(double a) { return isfinite(a); }
template <typename T> VX_HD T dsin(T a);
template <> VX_HD float dsin<float>(float a) { return sinf(a); }
template <> VX_HD double dsin<double>(double a) { return sin(a); }

// Reciprocal of x > 0: FP32 hardware estimate (1 ulp); FP64 hardware
// estimate refined by Newton steps to full precision.
template <typename T> VX_HD T frcp(T x);
template <> VX_HD float frcp<float>(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
template <> VX_HD double frcp<double>(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double y = __builtin_amdgcn_rcp(x);
#else
    double y = 1.0 / x;
#endif
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Quotient and square root of positive normal numbers, for the constants
// derived from per-voxel moduli and densities: FP32 takes the hardware
// reciprocal and square root (about 1 ulp, a few instructions instead of
// the correctly rounded sequences), FP64 the correctly rounded operations.
template <typename T> VX_HD T pdiv(T a, T b);
template <> VX_HD float pdiv<float>(float a, float b) { return a * frcp(b); }
template <> VX_HD double pdiv<double>(double a, double b) { return a / b; }
template <typename T> VX_HD T psqrt(T x);
template <> VX_HD float psqrt<float>(float x) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}
template <> VX_HD double psqrt<double>(double x) { return sqrt(x); }

// Series used on the common path, with the library functions as fallback
// outside their range.  Term counts make the truncation error smaller than
// half an ulp of the type over the whole fast range.
template <typename T> struct Series;
template <> struct Series<float> {
    static constexpr float kLogU = 0.01f;    // (|v| / w)^2 below which atan(t)/t is a polynomial
    static constexpr float kExpA2 = 0.01f;   // |w dt|^2 below which cos / sinc are polynomials
    static constexpr float kNormD = 1e-4f;   // |q|^2 - 1 below which 1/|q| is 1 - d/2 + 3d^2/8
};
template <> struct Series<double> {
    static constexpr double kLogU = 0.01;
    static constexpr double kExpA2 = 0.01;
    static constexpr double kNormD = 1e-6;
};

// atan(t)/t for u = t^2 < kLogU (alternating Taylor series 1 - u/3 + u^2/5 - ...).
template <typename T> VX_HD T atan_over_t(T u);
template <> VX_HD float atan_over_t<float>(float u) {
    float p = -1.0f / 7.0f;
    p = fmaf(p, u, 1.0f / 5.0f);
    p = fmaf(p, u, -1.0f / 3.0f);
    return fmaf(p, u, 1.0f);
}
template <> VX_HD double atan_over_t<double>(double u) {
    double p = -1.0 / 15.0;
    p = fma(p, u, 1.0 / 13.0);
    p = fma(p, u, -1.0 / 11.0);
    p = fma(p, u, 1.0 / 9.0);
    p = fma(p, u, -1.0 / 7.0);
    p = fma(p, u, 1.0 / 5.0);
    p = fma(p, u, -1.0 / 3.0);
    return fma(p, u, 1.0);
}

// cos(h) and sin(h) / (2 h) for a2 = (2 h)^2 < kExpA2 (Taylor in h^2 = a2/4).
template <typename T> VX_HD void half_angle_series(T a2, T *c, T *sk);
template <> VX_HD void half_angle_series<float>(float a2, float *c, float *sk) {
    const float h2 = 0.25f * a2;
    float pc = 1.0f / 24.0f;
    pc = fmaf(pc, h2, -0.5f);
    *c = fmaf(pc, h2, 1.0f);
    float ps = 1.0f / 120.0f;
    ps = fmaf(ps, h2, -1.0f / 6.0f);
    *sk = 0.5f * fmaf(ps, h2, 1.0f);
}
template <> VX_HD void half_angle_series<double>(double a2, double *c, double *sk) {
    const double h2 = 0.25 * a2;
    double pc = 1.0 / 40320.0;
    pc = fma(pc, h2, -1.0 / 720.0);
    pc = fma(pc, h2, 1.0 / 24.0);
    pc = fma(pc, h2, -0.5);
    *c = fma(pc, h2, 1.0);
    double ps = 1.0 / 362880.0;
    ps = fma(ps, h2, -1.0 / 5040.0);
    ps = fma(ps, h2, 1.0 / 120.0);
    ps = fma(ps, h2, -1.0 / 6.0);
    *sk = 0.5 * fma(ps, h2, 1.0);
}

// Element c of array base through a 32-bit byte offset from a uniform base,
// so the load/store addresses as SGPR base + one shared VGPR offset.
template <typename T>
VX_HD T ldc(const T *base, unsigned c) {
    return *(const T *)((const char *)base + (size_t)(c * (unsigned)sizeof(T)));
}
template <typename T>
VX_HD void stc(T *base, unsigned c, T v) {
    *(T *)((char *)base + (size_t)(c * (unsigned)sizeof(T))) = v;
}

// Kinematic quantities of one voxel that its bonds read.
template <typename T>
struct VoxKin {
    T ux, uy, uz;          // displacement from rest
    T qw, qx, qy, qz;      // orientation (body -> world)
    T vx, vy, vz;          // velocity P / m
    T wx, wy, wz;          // angular velocity phi / I
    T eps;                 // thermal strain at t_n
};

// Columns of the rotation matrix of a unit quaternion (body -> world), and
// its diagonal minus one (small near the identity, computed without
// cancellation).
template <typename T>
struct Rot {
    V3<T> c[3];
    T dm1[3];
};

template <typename T>
VX_HD Rot<T> rot_of(T w, T x, T y, T z) {
    Rot<T> R;
    const T two = T(2);
    R.dm1[0] = -two * (y * y + z * z);
    R.dm1[1] = -two * (x * x + z * z);
    R.dm1[2] = -two * (x * x + y * y);
    R.c[0] = {T(1) + R.dm1[0], two * (x * y + w * z), two * (x * z - w * y)};
    R.c[1] = {two * (x * y - w * z), T(1) + R.dm1[1], two * (y * z + w * x)};
    R.c[2] = {two * (x * z + w * y), two * (y * z - w * x), T(1) + R.dm1[2]};
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

// Constants of one bond.  On a cubic lattice (area l^2, I = l^4/12,
// J = l^4/6) Eq. 8-12 give b1 = a1, b2 = a1 l/2 and b3 = a1 l^2/6, and with
// the voxel inertia m l^2/6 the rotational damping coefficient of Eq. 35 is
// the translational one (Eq. 34) times l^2/6, so three numbers per material
// pair determine the bond.
template <typename T>
struct BondK {
    T a1, a2, ct;
};

// Lattice constants shared by every bond: l, l/2, l^2/6, l^2/3.
template <typename T>
struct LatK {
    T l, hl, l26, l23;
};

template <typename T>
VX_HD LatK<T> lat_consts(T l) {
    LatK<T> c;
    c.l = l; c.hl = T(0.5) * l; c.l26 = l * l / T(6); c.l23 = l * l / T(3);
    return c;
}

template <typename T>
VX_HD BondK<T> bond_k(const PairConst<T> &pc) {
    BondK<T> k;
    k.a1 = pc.a1; k.a2 = pc.a2; k.ct = pc.ct;
    return k;
}

// Rotation vector of q_A^-1 q_B (voxel 2's rotation relative to voxel 1, in
// voxel 1's body frame), on the short branch: 2 atan2(|v|, |w|) v / |v|.
template <typename T>
VX_HD void rel_rotvec(const VoxKin<T> &A, const VoxKin<T> &B, T th[3]) {
    const T rw = A.qw * B.qw + A.qx * B.qx + A.qy * B.qy + A.qz * B.qz;
    const T rx = A.qw * B.qx - A.qx * B.qw - A.qy * B.qz + A.qz * B.qy;
    const T ry = A.qw * B.qy + A.qx * B.qz - A.qy * B.qw - A.qz * B.qx;
    const T rz = A.qw * B.qz - A.qx * B.qy + A.qy * B.qx - A.qz * B.qw;
    const T aw = rw < T(0) ? -rw : rw;
    const T s2 = rx * rx + ry * ry + rz * rz;
    const T iw = frcp(aw);
    const T u = s2 * iw * iw;
    T k;
    if (u < Series<T>::kLogU) {
        k = T(2) * iw * atan_over_t(u);
    } else {
        const T s = dsqrt(s2);
        k = T(2) * datan2(s, aw) / s;
    }
    if (rw < T(0)) k = -k;
    th[0] = k * rx; th[1] = k * ry; th[2] = k * rz;
}

// One beam bond between voxel A (voxel 1, lower lattice index) and voxel B
// (voxel 2).  Co-rotational: the bond is expressed in the frame of voxel 1
// with its axis permuted onto +x (basis ex, ey, ez: columns of voxel 1's
// rotation), where only voxel 2's six displacements remain (reduced forces
// of Eq. 13-24, with the z-force sign of the full matrix Eq. 7).  The
// separation D_B - D_A is du + l e_axis (du the difference of
// displacements); ex_a, ey_a, ez_a are the axis components of the basis
// and exm1 = ex_a - 1, so the stretch X2 = ex.du + l (ex_a - 1) - l eps_mean
// never subtracts two numbers close to l.  (tx, ty, tz) is the relative
// rotation in the bond frame.  The result is rotated back to the world
// frame and bond damping (Eq. 33-35) is added.
template <typename T>
VX_HD BondOut<T> bond_core(const VoxKin<T> &A, const VoxKin<T> &B, const T du[3],
                                                const T d[3], const V3<T> &ex, const V3<T> &ey,
                                                const V3<T> &ez, T exm1, T ey_a, T ez_a, T tx, T ty, T tz,
                                                const BondK<T> &K, const LatK<T> &C) {
    // rest length stretched by the mean thermal strain (Eq. 40)
    const T X2 = ex.x * du[0] + ex.y * du[1] + ex.z * du[2] + C.l * (exm1 - T(0.5) * (A.eps + B.eps));
    const T Y2 = ey.x * du[0] + ey.y * du[1] + ey.z * du[2] + C.l * ey_a;
    const T Z2 = ez.x * du[0] + ez.y * du[1] + ez.z * du[2] + C.l * ez_a;
    const T b1 = K.a1, b2 = K.a1 * C.hl, b3 = K.a1 * C.l26, b3x2 = K.a1 * C.l23;
    // local nodal forces K u (u1 = 0)
    const T f2x = K.a1 * X2;
    const T f2y = b1 * Y2 - b2 * tz;
    const T f2z = b1 * Z2 + b2 * ty;
    const T m2x = K.a2 * tx;
    const T m2y = b2 * Z2 + b3x2 * ty;
    const T m2z = -b2 * Y2 + b3x2 * tz;
    const T m1x = -m2x;
    const T m1y = b2 * Z2 + b3 * ty;
    const T m1z = -b2 * Y2 + b3 * tz;
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
    const T cr = K.ct * C.l26;
    const T wax = A.wx + B.wx, way = A.wy + B.wy, waz = A.wz + B.wz;
    const T vrx = h * (B.vx - A.vx) + q4 * (d[1] * waz - d[2] * way);
    const T vry = h * (B.vy - A.vy) + q4 * (d[2] * wax - d[0] * waz);
    const T vrz = h * (B.vz - A.vz) + q4 * (d[0] * way - d[1] * wax);
    const T wrx = h * (B.wx - A.wx), wry = h * (B.wy - A.wy), wrz = h * (B.wz - A.wz);
    o.f2x -= K.ct * vrx; o.f2y -= K.ct * vry; o.f2z -= K.ct * vrz;
    o.m2x -= cr * wrx; o.m2y -= cr * wry; o.m2z -= cr * wrz;
    o.m1x += cr * wrx; o.m1y += cr * wry; o.m1z += cr * wrz;
    return o;
}

// Bond along lattice axis AX (compile-time).
template <typename T, int AX>
VX_HD BondOut<T> bond_eval(const VoxKin<T> &A, const Rot<T> &RA, const VoxKin<T> &B,
                                                const BondK<T> &K, const LatK<T> &C) {
    constexpr int A0 = AX, A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    const T du[3] = {B.ux - A.ux, B.uy - A.uy, B.uz - A.uz};
    T d[3] = {du[0], du[1], du[2]};
    d[AX] += C.l;
    T th[3];
    rel_rotvec(A, B, th);
    return bond_core(A, B, du, d, RA.c[A0], RA.c[A1], RA.c[A2], RA.dm1[A0], comp<AX>(RA.c[A1]),
                     comp<AX>(RA.c[A2]), th[A0], th[A1], th[A2], K, C);
}

// Bond along x (yaxis = false) or y (yaxis = true), chosen per lane.
template <typename T>
VX_HD BondOut<T> bond_eval_xy(const VoxKin<T> &A, const Rot<T> &RA, const VoxKin<T> &B,
                                                   const BondK<T> &K, const LatK<T> &C, bool yaxis) {
    const T du[3] = {B.ux - A.ux, B.uy - A.uy, B.uz - A.uz};
    T d[3] = {du[0], du[1], du[2]};
    d[0] += yaxis ? T(0) : C.l;
    d[1] += yaxis ? C.l : T(0);
    T th[3];
    rel_rotvec(A, B, th);
    const V3<T> ex = yaxis ? RA.c[1] : RA.c[0];
    const V3<T> ey = yaxis ? RA.c[2] : RA.c[1];
    const V3<T> ez = yaxis ? RA.c[0] : RA.c[2];
    const T exm1 = yaxis ? RA.dm1[1] : RA.dm1[0];
    const T ey_a = yaxis ? ey.y : ey.x, ez_a = yaxis ? ez.y : ez.x;
    const T tx = yaxis ? th[1] : th[0], ty = yaxis ? th[2] : th[1], tz = yaxis ? th[0] : th[2];
    return bond_core(A, B, du, d, ex, ey, ez, exm1, ey_a, ez_a, tx, ty, tz, K, C);
}

// Entry k of a per-channel table held in the step arguments (a select
// chain, so that the table stays in scalar registers).
template <typename T>
VX_HD T chan_pick(const Chan8<T> &c, int k) {
    // every member read at its fixed offset first: a conditional between two
    // members would select between their addresses
    const T v0 = c.v0, v1 = c.v1, v2 = c.v2, v3 = c.v3, v4 = c.v4, v5 = c.v5, v6 = c.v6, v7 = c.v7;
    T r = v0;
    if (k == 1) r = v1;
    if (k == 2) r = v2;
    if (k == 3) r = v3;
    if (k == 4) r = v4;
    if (k == 5) r = v5;
    if (k == 6) r = v6;
    if (k == 7) r = v7;
    return r;
}


// Strain of a voxel that follows no channel: its own signal, else the
// global one.  FP32 evaluates its own signal from the host-reduced phase
// 2 pi f t_n mod 2 pi.
template <typename T>
VX_HD T signal_strain(const StepArgs<T> &a, unsigned c, uint8_t fl, T cte) {
    T dT = a.dT_global;
    if (fl & FLAG_ACT) {
        if constexpr (sizeof(T) == 8) {
            dT = ldc(a.act_amp, c) * dsin<T>(a.wt + ldc(a.act_phase, c));
        } else {
            dT = ldc(a.act_amp, c) * dsin<T>(a.wt_red + ldc(a.act_phase, c));
        }
    }
    return cte * dT;
}

// Strain of a voxel at t_n: its channel's temperature (from the host), else
// signal_strain.
template <typename T>
VX_HD T voxel_strain(const StepArgs<T> &a, unsigned c, uint8_t fl, T cte) {
    if (fl & FLAG_CHAN) return cte * chan_pick(a.chan_dT, ldc(a.chan, c));
    return signal_strain(a, c, fl, cte);
}

// d eps / d phase and d eps / d amp of a voxel with its own actuation
// signal (FLAG_ACT) or of its channel's (FLAG_CHAN), at the same argument
// as voxel_strain.
template <typename T>
VX_HD void voxel_strain_d(const StepArgs<T> &a, const T *chan_dph, const T *chan_dam, unsigned c, uint8_t fl, T cte,
                          T *d_phase, T *d_amp) {
    if (fl & FLAG_CHAN) {
        const int k = ldc(a.chan, c);
        *d_phase = cte * chan_dph[k];
        *d_amp = cte * chan_dam[k];
        return;
    }
    const T amp = ldc(a.act_amp, c);
    T sn, cs;
    if constexpr (sizeof(T) == 8) {
        dsincos<T>(a.wt + ldc(a.act_phase, c), &sn, &cs);
    } else {
        dsincos<T>(a.wt_red + ldc(a.act_phase, c), &sn, &cs);
    }
    *d_phase = cte * amp * cs;
    *d_amp = cte * sn;
}

// Raw state words of one voxel.
template <typename T>
struct VoxRaw {
    T ux, uy, uz, qw, qx, qy, qz, px, py, pz, lx, ly, lz;
};

template <typename T>
VX_HD VoxRaw<T> load_raw(const T *__restrict__ s, long long st, unsigned c) {
    VoxRaw<T> r;
    r.ux = ldc(s + W_UX * st, c); r.uy = ldc(s + W_UY * st, c); r.uz = ldc(s + W_UZ * st, c);
    r.qw = ldc(s + W_QW * st, c); r.qx = ldc(s + W_QX * st, c);
    r.qy = ldc(s + W_QY * st, c); r.qz = ldc(s + W_QZ * st, c);
    r.px = ldc(s + W_PX * st, c); r.py = ldc(s + W_PY * st, c); r.pz = ldc(s + W_PZ * st, c);
    r.lx = ldc(s + W_LX * st, c); r.ly = ldc(s + W_LY * st, c); r.lz = ldc(s + W_LZ * st, c);
    return r;
}

template <typename T>
VX_HD void store_raw(T *__restrict__ o, long long st, unsigned c, T ux, T uy, T uz, T qw,
                                          T qx, T qy, T qz, T px, T py, T pz, T lx, T ly, T lz) {
    stc(o + W_UX * st, c, ux); stc(o + W_UY * st, c, uy); stc(o + W_UZ * st, c, uz);
    stc(o + W_QW * st, c, qw); stc(o + W_QX * st, c, qx); stc(o + W_QY * st, c, qy); stc(o + W_QZ * st, c, qz);
    stc(o + W_PX * st, c, px); stc(o + W_PY * st, c, py); stc(o + W_PZ * st, c, pz);
    stc(o + W_LX * st, c, lx); stc(o + W_LY * st, c, ly); stc(o + W_LZ * st, c, lz);
}

template <typename T>
VX_HD VoxKin<T> kin_of(const VoxRaw<T> &r, const MatConst<T> &mc, T eps) {
    VoxKin<T> k;
    k.ux = r.ux; k.uy = r.uy; k.uz = r.uz;
    k.qw = r.qw; k.qx = r.qx; k.qy = r.qy; k.qz = r.qz;
    k.vx = r.px * mc.inv_m; k.vy = r.py * mc.inv_m; k.vz = r.pz * mc.inv_m;
    k.wx = r.lx * mc.inv_I; k.wy = r.ly * mc.inv_I; k.wz = r.lz * mc.inv_I;
    k.eps = eps;
    return k;
}

template <typename T>
VX_HD VoxKin<T> load_kin(const T *__restrict__ s, long long stride, unsigned c,
                                              const MatConst<T> &mc, T eps) {
    return kin_of(load_raw(s, stride, c), mc, eps);
}

// Material constants of one voxel whose modulus E and density rho override
// the palette's (parameter mode): mass, inertia and the stiffness- and
// mass-dependent coefficients of a palette entry.  With I = m l^2/6 and the
// rotational stiffness E l^3/6, sqrt(I E l^3/6) = sqrt(m k_v) l^2/6, so one
// square root serves the three damping coefficients.
template <typename T>
VX_HD MatConst<T> mat_with(MatConst<T> mc, T E, T rho, T l, T zeta_slow, T zeta_col) {
    const T l26 = pdiv(l * l, T(6));
    mc.m = rho * l * l * l;
    mc.inv_m = pdiv(T(1), mc.m);
    mc.I = mc.m * l26;
    mc.inv_I = pdiv(T(1), mc.I);
    mc.E = E;
    mc.kv = E * l;
    const T s = psqrt(mc.m * mc.kv);
    mc.cg = T(2) * zeta_slow * s;
    mc.cgr = mc.cg * l26;
    mc.cfloor = T(2) * zeta_col * s;
    return mc;
}

// Bond constants from per-voxel moduli (Eq. 1, 2, 8-12, 34): g = 1/(2(1+nu))
// turns E into the shear modulus; m_min the smaller voxel mass.
template <typename T>
VX_HD BondK<T> bond_k_from_E(T EA, T EB, T gA, T gB, T m_min, T zeta_bond, const LatK<T> &C) {
    BondK<T> k;
    const T Ec = pdiv(T(2) * EA * EB, EA + EB);
    const T GA = EA * gA, GB = EB * gB;
    const T Gc = pdiv(T(2) * GA * GB, GA + GB);
    k.a1 = Ec * C.l;
    k.a2 = Gc * C.l * C.l26;
    k.ct = T(2) * zeta_bond * psqrt(m_min * k.a1);
    return k;
}

// Constants of cell c: the palette entry, or in parameter mode the entry
// with the cell's own modulus and density.
template <typename T>
VX_HD MatConst<T> mat_at(const StepArgs<T> &a, long long c, uint8_t m) {
    return a.E_cell ? mat_with(a.mats[m], a.E_cell[c], a.rho_cell[c], a.l, a.zeta_slow, a.zeta_col) : a.mats[m];
}

// Per-step environment of one voxel's update.
template <typename T>
struct UpdEnv {
    T dt, gravity, l;
    T z0;            // world z of the voxel's rest lower face minus half a voxel: origin_z + iz l
    int floor_on;
    T Fext[3];       // external force (FLAG_FORCED)
    T Fc[3];         // contact force (FLAG_CAND)
};

// Branch taken by the floor and friction logic (recorded for the adjoint).
enum : int { FR_NONE = 0, FR_HOLD = 1, FR_HALT_HOLD = 2, FR_HALT_SLIDE = 3, FR_SLIDE = 4 };

// Everything after the bond sum for one voxel: external force, gravity,
// ground damping, floor, contact, Coulomb friction (Eq. 36-38), then the
// synchronous "double Euler" update (Eq. 27-30) with the orientation
// advanced by the exact rotation w dt.  r is the voxel's state at t_n;
// returns the state at t_n+1 in o and the new flags in *nf_out.
template <typename T>
VX_HD void update_core(const UpdEnv<T> &e, uint8_t fl, const MatConst<T> &mc, T eps, const VoxRaw<T> &r, T Fx,
                       T Fy, T Fz, T Mx, T My, T Mz, VoxRaw<T> &o, uint8_t *nf_out, int *branch) {
    // One exit with every output assigned from scalars: early returns or
    // whole-struct copies of o make the compiler route it through private
    // memory.
    T ux = r.ux, uy = r.uy, uz = r.uz;
    const T qw = r.qw, qx = r.qx, qy = r.qy, qz = r.qz;
    T px = r.px, py = r.py, pz = r.pz;
    T lx = r.lx, ly = r.ly, lz = r.lz;
    T ow = qw, ox = qx, oy = qy, oz = qz;
    int br = FR_NONE;
    uint8_t nf = fl;
    if (fl & FLAG_FIXED) {
        px = py = pz = T(0);
        lx = ly = lz = T(0);
    } else {
        if (fl & FLAG_FORCED) { Fx += e.Fext[0]; Fy += e.Fext[1]; Fz += e.Fext[2]; }
        Fz -= mc.m * e.gravity;
        const T vx = px * mc.inv_m, vy = py * mc.inv_m, vz = pz * mc.inv_m;
        const T wx = lx * mc.inv_I, wy = ly * mc.inv_I, wz = lz * mc.inv_I;
        Fx -= vx * mc.cg; Fy -= vy * mc.cg; Fz -= vz * mc.cg;
        Mx -= wx * mc.cgr; My -= wy * mc.cgr; Mz -= wz * mc.cgr;
        T Fn = T(0);
        if (e.floor_on) {
            // s/2 - D_z with D_z = origin + (iz + 1/2) l + u_z; the half-voxel
            // terms cancel exactly
            const T pen = T(0.5) * e.l * eps - uz - e.z0;
            if (pen > T(0)) {
                Fn = mc.kv * pen - mc.cfloor * vz;
                if (Fn < T(0)) Fn = T(0);
                Fz += Fn;
            }
        }
        if (fl & FLAG_CAND) { Fx += e.Fc[0]; Fy += e.Fc[1]; Fz += e.Fc[2]; }
        if (e.floor_on) {
            if (Fn > T(0)) {
                const T Fl = dsqrt(Fx * Fx + Fy * Fy);
                bool done = false;
                if (nf & FLAG_STATIC) {
                    if (Fl <= mc.mu_s * Fn) {
                        Fx = T(0); Fy = T(0); px = T(0); py = T(0);
                        done = true;
                        br = FR_HOLD;
                    } else {
                        nf &= (uint8_t)~FLAG_STATIC;
                    }
                }
                if (!done) {
                    const T vl = dsqrt(vx * vx + vy * vy);
                    if (vl <= mc.mu_d * Fn * e.dt * mc.inv_m) {
                        px = T(0); py = T(0);
                        nf |= FLAG_STATIC;
                        if (Fl <= mc.mu_s * Fn) {
                            Fx = T(0); Fy = T(0);
                            br = FR_HALT_HOLD;
                        } else {
                            const T f = mc.mu_d * Fn / Fl;
                            Fx -= f * Fx; Fy -= f * Fy;
                            br = FR_HALT_SLIDE;
                        }
                    } else {
                        const T f = mc.mu_d * Fn / vl;
                        Fx -= f * vx; Fy -= f * vy;
                        br = FR_SLIDE;
                    }
                }
            } else {
                nf &= (uint8_t)~FLAG_STATIC;
            }
        }
        // integrate
        const T dt = e.dt;
        px += Fx * dt; py += Fy * dt; pz += Fz * dt;
        const T nvx = px * mc.inv_m, nvy = py * mc.inv_m, nvz = pz * mc.inv_m;
        ux += nvx * dt; uy += nvy * dt; uz += nvz * dt;
        lx += Mx * dt; ly += My * dt; lz += Mz * dt;
        const T rx = lx * mc.inv_I * dt, ry = ly * mc.inv_I * dt, rz = lz * mc.inv_I * dt;
        const T a2 = rx * rx + ry * ry + rz * rz;
        T dw, sk;
        if (a2 < Series<T>::kExpA2) {
            half_angle_series(a2, &dw, &sk);
        } else {
            const T ang = dsqrt(a2);
            T sn, cs;
            dsincos(T(0.5) * ang, &sn, &cs);
            dw = cs;
            sk = sn / ang;
        }
        const T dx = sk * rx, dy = sk * ry, dz = sk * rz;
        // dq * q, then normalise
        const T nw = dw * qw - dx * qx - dy * qy - dz * qz;
        const T nx = dw * qx + dx * qw + dy * qz - dz * qy;
        const T ny = dw * qy - dx * qz + dy * qw + dz * qx;
        const T nz = dw * qz + dx * qy - dy * qx + dz * qw;
        const T n2 = nw * nw + nx * nx + ny * ny + nz * nz;
        const T dn = n2 - T(1);
        T inv;
        if (dn < Series<T>::kNormD && dn > -Series<T>::kNormD) {
            inv = fma(dn, fma(dn, T(0.375), T(-0.5)), T(1));
        } else {
            inv = T(1) / dsqrt(n2);
        }
        ow = nw * inv; ox = nx * inv; oy = ny * inv; oz = nz * inv;
    }
    o.ux = ux; o.uy = uy; o.uz = uz;
    o.qw = ow; o.qx = ox; o.qy = oy; o.qz = oz;
    o.px = px; o.py = py; o.pz = pz;
    o.lx = lx; o.ly = ly; o.lz = lz;
    *nf_out = nf;
    *branch = br;
}

// Voxel update of cell c from its bond sums: gathers the per-voxel inputs
// of update_core, writes the new state and flags, flags non-finite values
// and tracks the largest squared speed in *vmax_local.
template <typename T>
__device__ __forceinline__ UpdEnv<T> upd_env(const StepArgs<T> &a, unsigned c, uint8_t fl) {
    UpdEnv<T> e;
    e.dt = a.dt; e.gravity = a.gravity; e.l = a.l; e.floor_on = a.floor_on;
    const unsigned nxy = (unsigned)a.nx * (unsigned)a.ny;
    e.z0 = a.origin_z + T((int)(c / nxy)) * a.l;
    e.Fext[0] = e.Fext[1] = e.Fext[2] = T(0);
    e.Fc[0] = e.Fc[1] = e.Fc[2] = T(0);
    if (fl & FLAG_FORCED) {
        int lo = 0, hi = a.n_forced - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((unsigned)a.forced_cells[mid] < c) lo = mid + 1; else hi = mid;
        }
        e.Fext[0] = a.forced_F[3 * lo]; e.Fext[1] = a.forced_F[3 * lo + 1]; e.Fext[2] = a.forced_F[3 * lo + 2];
    }
    if (fl & FLAG_CAND) {
        const long long st = a.stride;
        e.Fc[0] = ldc(a.contact_F, c); e.Fc[1] = ldc(a.contact_F + st, c); e.Fc[2] = ldc(a.contact_F + 2 * st, c);
    }
    return e;
}

// store(c, o) writes the new state words of cell c.
template <typename T, typename Store>
__device__ __forceinline__ void voxel_update(const StepArgs<T> &a, unsigned c, uint8_t fl,
                                             const MatConst<T> &mc, T eps, const VoxRaw<T> &r, T Fx,
                                             T Fy, T Fz, T Mx, T My, T Mz, T *vmax_local, const Store &store) {
    const UpdEnv<T> e = upd_env(a, c, fl);
    VoxRaw<T> o;
    uint8_t nf;
    int branch;
    update_core(e, fl, mc, eps, r, Fx, Fy, Fz, Mx, My, Mz, o, &nf, &branch);
    store(c, o);
    stc(a.flags_out, c, nf);
    if (fl & FLAG_FIXED) return;
    // a non-finite momentum reaches the displacement, and a non-finite
    // angular momentum the orientation, in the same update
    const bool ok = dfinite(o.ux) && dfinite(o.uy) && dfinite(o.uz) && dfinite(o.qw) && dfinite(o.qx) &&
                    dfinite(o.qy) && dfinite(o.qz) && dfinite(o.px) && dfinite(o.py) && dfinite(o.pz) &&
                    dfinite(o.lx) && dfinite(o.ly) && dfinite(o.lz);
    if (!ok) atomicOr(a.err_flag, 1u);
    const T nvx = o.px * mc.inv_m, nvy = o.py * mc.inv_m, nvz = o.pz * mc.inv_m;
    const T sp2 = nvx * nvx + nvy * nvy + nvz * nvz;
    if (sp2 > *vmax_local) *vmax_local = sp2;
}

template <typename T>
__device__ __forceinline__ void voxel_update(const StepArgs<T> &a, unsigned c, uint8_t fl,
                                             const MatConst<T> &mc, T eps, const VoxRaw<T> &r, T Fx,
                                             T Fy, T Fz, T Mx, T My, T Mz, T *vmax_local) {
    voxel_update(a, c, fl, mc, eps, r, Fx, Fy, Fz, Mx, My, Mz, vmax_local, [&](unsigned cc, const VoxRaw<T> &o) {
        store_raw(a.s_out, a.stride, cc, o.ux, o.uy, o.uz, o.qw, o.qx, o.qy, o.qz, o.px, o.py, o.pz, o.lx, o.ly,
                  o.lz);
    });
}

// Wavefront maximum of the squared speed v2, then one atomic per wave of the
// speed into the device-wide maximum (non-negative doubles order like their
// bit patterns).
template <typename T>
__device__ __forceinline__ void wave_vmax(unsigned long long *dst, T v) {
    for (int off = 32; off > 0; off >>= 1) {
        const T o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    if ((threadIdx.x & 63) == 0 && v > T(0)) {
        const double d = sqrt((double)v);
        atomicMax(dst, (unsigned long long)__double_as_longlong(d));
    }
}

// Collision motion bookkeeping of one step, by one thread after the step
// kernel: a rebuild that ran at the step's start (flag still set) is
// closed, the largest speed of the step (read and cleared) times dt is
// accumulated, and the flag is set for the next step once twice the
// accumulated motion reaches the threshold (or always).  Every word is read
// before any is written, so the thread waits on memory once.  Returns the
// flag as found: whether a rebuild ran at the step's start.
__device__ __forceinline__ unsigned motion_update(Scalars *sc, double dt) {
    const unsigned flag = sc->rebuild_flag, every = sc->every;
    const double macc = sc->macc, threshold = sc->threshold;
    const unsigned long long rebuilds = sc->rebuilds;
    const double v = __longlong_as_double((long long)atomicExch(&sc->vmax_bits, 0ull));
    const double acc = (flag ? 0.0 : macc) + v * dt;
    if (flag) sc->rebuilds = rebuilds + 1ull;
    sc->macc = acc;
    sc->rebuild_flag = (every || 2.0 * acc >= threshold) ? 1u : 0u;
    return flag;
}

}  // namespace vx
