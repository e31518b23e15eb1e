// Reverse of one split step, in three passes mirroring the forward:
//   1. per voxel: VJP of the update (environment, friction, integration),
//      giving the adjoint of x_n through the voxel's own state and the
//      adjoints of its bond sums;
//   2. per bond and axis: VJP of the bond force, writing both ends' adjoints
//      and the moduli adjoints to a record;
//   3. per voxel: gathers its at most six records in the forward's fixed
//      order, completes the adjoint of x_n and accumulates the parameter
//      gradients in FP64.
// No atomics: every output word has one writer, so the reverse pass is as
// deterministic as the forward one.
#include "vx_adjoint.hpp"
#include "vx_launch.hpp"

namespace vx {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_adj_update(StepArgs<T> a, AdjArgs<T> g) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint8_t m = a.mat[c];
    if (m == 0) return;
    const long long st = a.stride;
    const MatConst<T> mc = mat_at(a, c, m);
    const uint8_t fl = a.flags[c];
    const T eps = voxel_strain(a, (unsigned)c, fl, mc.cte);
    const VoxRaw<T> r = load_raw(a.s_in, st, (unsigned)c);
    const VoxRaw<T> lam = load_raw(g.lam_in, st, (unsigned)c);
    const T *fm = g.fm;
    const UpdEnv<T> e = upd_env(a, (unsigned)c, fl);
    const UpdAdj<T> ad = update_vjp(e, fl, mc, eps, r, fm[c], fm[st + c], fm[2 * st + c], fm[3 * st + c],
                                    fm[4 * st + c], fm[5 * st + c], lam);
    store_raw(g.lam_out, st, (unsigned)c, ad.r.ux, ad.r.uy, ad.r.uz, ad.r.qw, ad.r.qx, ad.r.qy, ad.r.qz, ad.r.px,
              ad.r.py, ad.r.pz, ad.r.lx, ad.r.ly, ad.r.lz);
    T *gfm = g.gfm;
    gfm[c] = ad.Fx; gfm[st + c] = ad.Fy; gfm[2 * st + c] = ad.Fz;
    gfm[3 * st + c] = ad.Mx; gfm[4 * st + c] = ad.My; gfm[5 * st + c] = ad.Mz;
    // kv = E l; cg, cgr, cfloor are proportional to sqrt(E m) (I = m l^2/6);
    // inv_m = 1/m, inv_I = 6/(m l^2)
    const T gd = ad.cg * mc.cg + ad.cgr * mc.cgr + ad.cfloor * mc.cfloor;
    const T gE = ad.kv * a.l + gd / (T(2) * mc.E);
    const T gm = ad.m - (ad.inv_m * mc.inv_m + ad.inv_I * mc.inv_I) / mc.m + gd / (T(2) * mc.m);
    g.gloc[c] = ad.eps;
    g.gloc[st + c] = gE;
    g.gloc[2 * st + c] = gm;
}

template <typename T, int AX>
__global__ void __launch_bounds__(256) k_adj_bonds(StepArgs<T> a, AdjArgs<T> g) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint8_t ma = a.mat[c];
    if (ma == 0) return;
    const long long nxy = (long long)a.nx * a.ny;
    long long cn;
    if (AX == 0) {
        if ((int)(c % a.nx) + 1 >= a.nx) return;
        cn = c + 1;
    } else if (AX == 1) {
        if ((int)((c / a.nx) % a.ny) + 1 >= a.ny) return;
        cn = c + a.nx;
    } else {
        if ((int)(c / nxy) + 1 >= a.nz) return;
        cn = c + nxy;
    }
    const uint8_t mb = a.mat[cn];
    if (mb == 0) return;
    const long long st = a.stride;
    const MatConst<T> A = mat_at(a, c, ma), B = mat_at(a, cn, mb);
    const T ea = voxel_strain(a, (unsigned)c, a.flags[c], A.cte);
    const T eb = voxel_strain(a, (unsigned)cn, a.flags[cn], B.cte);
    const VoxKin<T> ka = load_kin(a.s_in, st, (unsigned)c, A, ea);
    const VoxKin<T> kb = load_kin(a.s_in, st, (unsigned)cn, B, eb);
    const LatK<T> C = lat_consts(a.l);
    const T EA = a.E_cell[c], EB = a.E_cell[cn];
    const BondK<T> K = bond_k_from_E(EA, EB, A.gfac, B.gfac, A.m < B.m ? A.m : B.m, a.zeta_bond, C);
    // the bond adds F2 to voxel 2, -F2 to voxel 1, M1 and M2
    const T *gfm = g.gfm;
    const T gF[3] = {gfm[cn] - gfm[c], gfm[st + cn] - gfm[st + c], gfm[2 * st + cn] - gfm[2 * st + c]};
    const T gM1[3] = {gfm[3 * st + c], gfm[4 * st + c], gfm[5 * st + c]};
    const T gM2[3] = {gfm[3 * st + cn], gfm[4 * st + cn], gfm[5 * st + cn]};
    const BondAdj<T> ad = bond_vjp<T, AX>(ka, kb, K, C, gF, gM1, gM2);
    T gEA, gEB;
    bond_k_from_E_vjp(EA, EB, A.gfac, B.gfac, K, ad.a1, ad.a2, ad.ct, C, &gEA, &gEB);
    // ct = 2 zeta sqrt(m_min a1): the lighter voxel's mass (B on a tie, as
    // the forward picks it)
    const T mmin = A.m < B.m ? A.m : B.m;
    const T gmmin = ad.ct * K.ct / (T(2) * mmin);
    const T gmA = A.m < B.m ? gmmin : T(0), gmB = A.m < B.m ? T(0) : gmmin;
    T *r = g.rec + (long long)AX * kAdjRecWords * st + c;
    const KinAdj<T> *ends[2] = {&ad.A, &ad.B};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const KinAdj<T> &k = *ends[e];
        T *o = r + (long long)e * 14 * st;
        o[0 * st] = k.ux; o[1 * st] = k.uy; o[2 * st] = k.uz;
        o[3 * st] = k.qw; o[4 * st] = k.qx; o[5 * st] = k.qy; o[6 * st] = k.qz;
        o[7 * st] = k.vx; o[8 * st] = k.vy; o[9 * st] = k.vz;
        o[10 * st] = k.wx; o[11 * st] = k.wy; o[12 * st] = k.wz;
        o[13 * st] = k.eps;
    }
    r[28 * st] = gEA;
    r[29 * st] = gEB;
    r[30 * st] = gmA;
    r[31 * st] = gmB;
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_gather(StepArgs<T> a, AdjArgs<T> g) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint8_t m = a.mat[c];
    if (m == 0) return;
    const long long st = a.stride;
    const long long nxy = (long long)a.nx * a.ny;
    const int idx[3] = {(int)(c % a.nx), (int)((c / a.nx) % a.ny), (int)(c / nxy)};
    const int dim[3] = {a.nx, a.ny, a.nz};
    const long long step[3] = {1, a.nx, nxy};
    // (u, q, v, w, eps) adjoints of this voxel's bond inputs
    T k[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) k[i] = T(0);
    T gE = g.gloc[st + c];
    T gm = g.gloc[2 * st + c];
    // fixed order as in the forward sum: -x, +x, -y, +y, -z, +z
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const T *rb = g.rec + (long long)ax * kAdjRecWords * st;
        if (idx[ax] > 0 && a.mat[c - step[ax]] != 0) {   // voxel 2 of the bond at c - step
            const T *o = rb + 14 * st + (c - step[ax]);
#pragma unroll
            for (int i = 0; i < 14; ++i) k[i] += o[i * st];
            gE += rb[29 * st + (c - step[ax])];
            gm += rb[31 * st + (c - step[ax])];
        }
        if (idx[ax] + 1 < dim[ax] && a.mat[c + step[ax]] != 0) {   // voxel 1 of the bond at c
            const T *o = rb + c;
#pragma unroll
            for (int i = 0; i < 14; ++i) k[i] += o[i * st];
            gE += rb[28 * st + c];
            gm += rb[30 * st + c];
        }
    }
    const MatConst<T> mc = mat_at(a, c, m);
    VoxRaw<T> lam = load_raw(g.lam_out, st, (unsigned)c);
    lam.ux += k[0]; lam.uy += k[1]; lam.uz += k[2];
    lam.qw += k[3]; lam.qx += k[4]; lam.qy += k[5]; lam.qz += k[6];
    // v = P / m, w = L / I
    lam.px += k[7] * mc.inv_m; lam.py += k[8] * mc.inv_m; lam.pz += k[9] * mc.inv_m;
    lam.lx += k[10] * mc.inv_I; lam.ly += k[11] * mc.inv_I; lam.lz += k[12] * mc.inv_I;
    store_raw(g.lam_out, st, (unsigned)c, lam.ux, lam.uy, lam.uz, lam.qw, lam.qx, lam.qy, lam.qz, lam.px, lam.py,
              lam.pz, lam.lx, lam.ly, lam.lz);
    // the bonds read v = P inv_m and w = L inv_I of this voxel
    const VoxRaw<T> r = load_raw(a.s_in, st, (unsigned)c);
    const T g_inv_m = k[7] * r.px + k[8] * r.py + k[9] * r.pz;
    const T g_inv_I = k[10] * r.lx + k[11] * r.ly + k[12] * r.lz;
    gm -= (g_inv_m * mc.inv_m + g_inv_I * mc.inv_I) / mc.m;
    g.g_E[c] += (double)gE;
    g.g_rho[c] += (double)gm * ((double)a.l * (double)a.l * (double)a.l);
    const uint8_t fl = a.flags[c];
    if (fl & FLAG_ACT) {
        const T geps = g.gloc[c] + k[13];
        T dph, dam;
        voxel_strain_d(a, (unsigned)c, mc.cte, &dph, &dam);
        g.g_phase[c] += (double)(geps * dph);
        g.g_amp[c] += (double)(geps * dam);
    }
}

}  // namespace

template <typename T>
hipError_t launch_adjoint_step(const StepArgs<T> &a, const AdjArgs<T> &g, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_adj_update<T><<<blocks, 256, 0, s>>>(a, g);
    k_adj_bonds<T, 0><<<blocks, 256, 0, s>>>(a, g);
    k_adj_bonds<T, 1><<<blocks, 256, 0, s>>>(a, g);
    k_adj_bonds<T, 2><<<blocks, 256, 0, s>>>(a, g);
    k_adj_gather<T><<<blocks, 256, 0, s>>>(a, g);
    return hipGetLastError();
}

template hipError_t launch_adjoint_step<float>(const StepArgs<float> &, const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_step<double>(const StepArgs<double> &, const AdjArgs<double> &, hipStream_t);

}  // namespace vx
