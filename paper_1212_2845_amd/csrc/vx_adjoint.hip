// Reverse of one split step.  k_adj_update applies, per voxel, the VJP of
// the update (environment, friction, integration): it gives the adjoint of
// x_n through the voxel's own state, the adjoints of its bond sums, and the
// update's adjoints of the voxel's strain, modulus and mass.  With
// self-collision the contact forces' reverse (vx_collide.hip) adds to
// these next.  The bond pass and the gather that complete the adjoint of
// x_n and accumulate the parameter gradients run as one LDS-tiled launch
// (vx_adjoint_fused.hip).
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
    const long long st = a.stride;
    const unsigned cu = (unsigned)c;
    // an empty cell stops at its material byte (on a sparse lattice whole
    // waves do); every other word a filled cell contributes is loaded
    // before any is used, so that the loads are in flight together instead
    // of waiting on the flags, then on the parameters, then on the signal
    const uint8_t m = a.mat[c];
    if (m == 0) return;
    const uint8_t fl = a.flags[c];
    const VoxRaw<T> r = load_raw(a.s_in, st, cu);
    const VoxRaw<T> lam = load_raw(g.lam_in, st, cu);
    const T *fm = g.fm;
    const T f0 = ldc(fm, cu), f1 = ldc(fm + st, cu), f2 = ldc(fm + 2 * st, cu);
    const T f3 = ldc(fm + 3 * st, cu), f4 = ldc(fm + 4 * st, cu), f5 = ldc(fm + 5 * st, cu);
    const T amp = ldc(a.act_amp, cu), phase = ldc(a.act_phase, cu);
    const uint8_t ch = ldc(a.chan, cu);
    T Ec = T(0), rhoc = T(0);
    if (a.E_cell) { Ec = ldc(a.E_cell, cu); rhoc = ldc(a.rho_cell, cu); }
    const MatConst<T> mc = a.E_cell ? mat_with(a.mats[m], Ec, rhoc, a.l, a.zeta_slow, a.zeta_col) : a.mats[m];
    // the strain as voxel_strain takes it, from the words above
    T dT = a.dT_global;
    if (fl & FLAG_CHAN) {
        dT = chan_pick(a.chan_dT, ch);
    } else if (fl & FLAG_ACT) {
        if constexpr (sizeof(T) == 8) dT = amp * dsin<T>(a.wt + phase);
        else dT = amp * dsin<T>(a.wt_red + phase);
    }
    const T eps = mc.cte * dT;
    const UpdEnv<T> e = upd_env(a, cu, fl);
    const UpdAdj<T> ad = update_vjp(e, fl, mc, eps, r, f0, f1, f2, f3, f4, f5, lam);
    store_raw(g.lam_out, st, (unsigned)c, ad.r.ux, ad.r.uy, ad.r.uz, ad.r.qw, ad.r.qx, ad.r.qy, ad.r.qz, ad.r.px,
              ad.r.py, ad.r.pz, ad.r.lx, ad.r.ly, ad.r.lz);
    T *gfm = g.gfm;
    gfm[c] = ad.Fx; gfm[st + c] = ad.Fy; gfm[2 * st + c] = ad.Fz;
    gfm[3 * st + c] = ad.Mx; gfm[4 * st + c] = ad.My; gfm[5 * st + c] = ad.Mz;
    // kv = E l; cg, cgr, cfloor are proportional to sqrt(E m) (I = m l^2/6);
    // inv_m = 1/m, inv_I = 6/(m l^2)
    const T gd = ad.cg * mc.cg + ad.cgr * mc.cgr + ad.cfloor * mc.cfloor;
    const T gE = ad.kv * a.l + pdiv(gd, T(2) * mc.E);
    const T gm = ad.m - (ad.inv_m * mc.inv_m + ad.inv_I * mc.inv_I) * mc.inv_m + gd * T(0.5) * mc.inv_m;
    g.gloc[c] = ad.eps;
    g.gloc[st + c] = gE;
    g.gloc[2 * st + c] = gm;
}

}  // namespace

template <typename T>
hipError_t launch_adjoint_step(const StepArgs<T> &a, const AdjArgs<T> &g, const CollideArgs *c, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_adj_update<T><<<blocks, 256, 0, s>>>(a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (c) {
        e = launch_adjoint_contact<T>(a, *c, g, s);
        if (e != hipSuccess) return e;
    }
    return launch_adjoint_fused<T>(a, g, s);
}

template hipError_t launch_adjoint_step<float>(const StepArgs<float> &, const AdjArgs<float> &, const CollideArgs *,
                                               hipStream_t);
template hipError_t launch_adjoint_step<double>(const StepArgs<double> &, const AdjArgs<double> &, const CollideArgs *,
                                                hipStream_t);

}  // namespace vx
