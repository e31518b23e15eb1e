// Fused reverse of the bond pass and the gather: one launch per reverse step
// after k_adj_update has produced every voxel's bond-sum adjoint.
//
// A workgroup owns a TX x TY column of cells and marches up a chunk of z
// slabs, like the forward fused kernel.  Per slab, the own cells and a
// one-cell ring are staged in LDS (kinematics at x_n, modulus, mass, shear
// factor, bond-sum adjoint).  Each thread evaluates the VJP of its voxel's
// +x, +y and +z bonds, keeps its own end's adjoint in registers and hands
// the other end's 16 words over: through LDS for x and y, in registers to
// the next slab for z.  Threads on the tile's low x and y faces also
// evaluate the bonds entering from the ring (only the inner end is kept),
// and the bond entering the chunk from below is evaluated once per column.
// No per-bond record reaches HBM and no atomics are used.  Every word a
// cell contributes (material, flags, modulus, density, signal, state, bond-
// sum adjoint) is loaded without waiting on another, and the next slab is
// staged in LDS between the bond pass and the gather.
#include "vx_adjoint.hpp"
#include "vx_launch.hpp"

namespace vx {

namespace {

constexpr int kAdjTX = 32, kAdjTY = 8;
constexpr int kAdjXcds = 8;
constexpr int kAdjKin = 14;   // u (3), q (4), v (3), w (3), eps
constexpr int kEnd = 16;      // one bond end's adjoint: kinematics (14), modulus, mass

// One cell as a bond end in the reverse pass.
template <typename T>
struct AdjCell {
    uint8_t m;
    VoxKin<T> k;
    T E, mass, gfac;
    T gf[6];      // adjoint of the cell's bond force and moment sums
};

template <typename T, int NR, int NBX, int NBY>
struct AdjSmem {
    T kin[kAdjKin][NR];
    T par[3][NR];     // modulus, mass, shear factor
    T gfm[6][NR];
    T rx[kEnd][NBX];  // voxel-2 ends of the x bonds of the slab
    T ry[kEnd][NBY];
    uint8_t mat[NR];
};

// Every word one cell contributes to the reverse pass, loaded without
// waiting on any of them (also for an empty cell, whose words exist and are
// ignored), so that the loads of a slab are in flight together.
template <typename T>
struct AdjPre {
    uint8_t m, fl, ch;
    T E, rho, amp, phase;
    VoxRaw<T> r;
    T gf[6];
};

template <typename T>
__device__ __forceinline__ void issue_adj(const StepArgs<T> &a, const AdjArgs<T> &g, unsigned c, AdjPre<T> &p) {
    p.m = ldc(a.mat, c);
    p.fl = ldc(a.flags, c);
    p.E = a.E_cell ? ldc(a.E_cell, c) : T(0);
    p.rho = a.rho_cell ? ldc(a.rho_cell, c) : T(0);
    p.amp = ldc(a.act_amp, c);
    p.phase = ldc(a.act_phase, c);
    p.ch = ldc(a.chan, c);
    p.r = load_raw(a.s_in, a.stride, c);
#pragma unroll
    for (int i = 0; i < 6; ++i) p.gf[i] = ldc(g.gfm + i * a.stride, c);
}

// Strain of a cell from its prefetched signal: the same expression as
// voxel_strain.
template <typename T>
__device__ __forceinline__ T strain_of(const StepArgs<T> &a, const T *chan_dT, uint8_t fl, T cte, T amp, T phase,
                                       int ch) {
    T dT = a.dT_global;
    if (fl & FLAG_CHAN) {
        dT = chan_dT[ch];
    } else if (fl & FLAG_ACT) {
        if constexpr (sizeof(T) == 8) {
            dT = amp * dsin<T>(a.wt + phase);
        } else {
            dT = amp * dsin<T>(a.wt_red + phase);
        }
    }
    return cte * dT;
}

template <typename T>
__device__ __forceinline__ void finish_adj(const StepArgs<T> &a, const T *chan_dT, const AdjPre<T> &p,
                                           AdjCell<T> &o) {
    o.m = p.m;
    if (!p.m) return;
    const MatConst<T> mc = a.E_cell ? mat_with(a.mats[p.m], p.E, p.rho, a.l, a.zeta_slow, a.zeta_col) : a.mats[p.m];
    const T eps = strain_of(a, chan_dT, p.fl, mc.cte, p.amp, p.phase, p.ch);
    o.k = kin_of(p.r, mc, eps);
    o.E = mc.E; o.mass = mc.m; o.gfac = mc.gfac;
#pragma unroll
    for (int i = 0; i < 6; ++i) o.gf[i] = p.gf[i];
}

template <typename T>
__device__ __forceinline__ void load_cell(const StepArgs<T> &a, const AdjArgs<T> &g, const T *chan_dT, unsigned c,
                                          AdjCell<T> &o) {
    AdjPre<T> p;
    issue_adj(a, g, c, p);
    finish_adj(a, chan_dT, p, o);
}

template <typename T, typename S>
__device__ __forceinline__ void put_cell(S &sm, int slot, const AdjCell<T> &o) {
    const T *k = &o.k.ux;
#pragma unroll
    for (int i = 0; i < kAdjKin; ++i) sm.kin[i][slot] = k[i];
    sm.par[0][slot] = o.E; sm.par[1][slot] = o.mass; sm.par[2][slot] = o.gfac;
#pragma unroll
    for (int i = 0; i < 6; ++i) sm.gfm[i][slot] = o.gf[i];
}

template <typename T, typename S>
__device__ __forceinline__ AdjCell<T> get_cell(const S &sm, int slot) {
    AdjCell<T> o;
    o.m = sm.mat[slot];
    T *k = &o.k.ux;
#pragma unroll
    for (int i = 0; i < kAdjKin; ++i) k[i] = sm.kin[i][slot];
    o.E = sm.par[0][slot]; o.mass = sm.par[1][slot]; o.gfac = sm.par[2][slot];
#pragma unroll
    for (int i = 0; i < 6; ++i) o.gf[i] = sm.gfm[i][slot];
    return o;
}

// VJP of the bond from A (voxel 1) to B (voxel 2) along AX: both ends'
// adjoints of (u, q, v, w, eps), modulus and mass.
template <typename T, int AX>
__device__ __forceinline__ void bond_ends(const AdjCell<T> &A, const AdjCell<T> &B, T zeta_bond, const LatK<T> &C,
                                          T ea[kEnd], T eb[kEnd]) {
    const T mmin = A.mass < B.mass ? A.mass : B.mass;
    const BondK<T> K = bond_k_from_E(A.E, B.E, A.gfac, B.gfac, mmin, zeta_bond, C);
    const T gF[3] = {B.gf[0] - A.gf[0], B.gf[1] - A.gf[1], B.gf[2] - A.gf[2]};
    const T gM1[3] = {A.gf[3], A.gf[4], A.gf[5]};
    const T gM2[3] = {B.gf[3], B.gf[4], B.gf[5]};
    const BondAdj<T> ad = bond_vjp<T, AX>(A.k, B.k, K, C, gF, gM1, gM2);
    const T *pa = &ad.A.ux, *pb = &ad.B.ux;
#pragma unroll
    for (int i = 0; i < kAdjKin; ++i) { ea[i] = pa[i]; eb[i] = pb[i]; }
    bond_k_from_E_vjp(A.E, B.E, A.gfac, B.gfac, K, ad.a1, ad.a2, ad.ct, C, &ea[14], &eb[14]);
    // bond damping takes the lighter mass; on a tie, where the smaller mass
    // has no derivative, each voxel takes half (the mean of the two
    // one-sided derivatives)
    const T gmmin = ad.ct * pdiv(K.ct, T(2) * mmin);
    const T wa = A.mass < B.mass ? T(1) : (B.mass < A.mass ? T(0) : T(0.5));
    ea[15] = wa * gmmin;
    eb[15] = (T(1) - wa) * gmmin;
}

// Adjoint of x_n of cell c from its direct part (k_adj_update) and the sum k
// of its bond ends; FP64 accumulation of the parameter gradients.
template <typename T>
__device__ __forceinline__ void finish_voxel(const StepArgs<T> &a, const AdjArgs<T> &g, const T (*chan)[kMaxChan],
                                             unsigned c, uint8_t m,
                                             const T k[kEnd]) {
    const long long st = a.stride;
    const MatConst<T> mc = mat_at(a, (long long)c, m);
    VoxRaw<T> lam = load_raw(g.lam_out, st, c);
    lam.ux += k[0]; lam.uy += k[1]; lam.uz += k[2];
    lam.qw += k[3]; lam.qx += k[4]; lam.qy += k[5]; lam.qz += k[6];
    lam.px += k[7] * mc.inv_m; lam.py += k[8] * mc.inv_m; lam.pz += k[9] * mc.inv_m;
    lam.lx += k[10] * mc.inv_I; lam.ly += k[11] * mc.inv_I; lam.lz += k[12] * mc.inv_I;
    store_raw(g.lam_out, st, c, lam.ux, lam.uy, lam.uz, lam.qw, lam.qx, lam.qy, lam.qz, lam.px, lam.py, lam.pz,
              lam.lx, lam.ly, lam.lz);
    // the bonds read v = P inv_m and w = L inv_I of this voxel
    const VoxRaw<T> r = load_raw(a.s_in, st, c);
    const T g_inv_m = k[7] * r.px + k[8] * r.py + k[9] * r.pz;
    const T g_inv_I = k[10] * r.lx + k[11] * r.ly + k[12] * r.lz;
    const T gE = ldc(g.gloc + st, c) + k[14];
    const T gm = ldc(g.gloc + 2 * st, c) + k[15] - (g_inv_m * mc.inv_m + g_inv_I * mc.inv_I) * mc.inv_m;
    g.g_E[c] += (double)gE;
    g.g_rho[c] += (double)gm * ((double)a.l * (double)a.l * (double)a.l);
    const uint8_t fl = ldc(a.flags, c);
    if (fl & (FLAG_ACT | FLAG_CHAN)) {
        const T geps = ldc(g.gloc, c) + k[13];
        T dph, dam;
        voxel_strain_d(a, chan[1], chan[2], c, fl, mc.cte, &dph, &dam);
        g.g_phase[c] += (double)(geps * dph);
        g.g_amp[c] += (double)(geps * dam);
    }
}

struct AdjGrid {
    int tiles_x, tiles_y, chunks, zc;
};

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) k_adj_fused(StepArgs<T> a, AdjArgs<T> g, AdjGrid fg) {
    static_assert(2 * (TX + TY) <= TX * TY, "ring must fit one cell per thread");
    constexpr int RW = TX + 2, NR = (TX + 2) * (TY + 2), NBX = (TX + 1) * TY, NBY = TX * (TY + 1);
    __shared__ AdjSmem<T, NR, NBX, NBY> sm;
    // the channels' temperatures and their derivatives at t_n, staged once
    // (the step arguments' copies are not kept in registers)
    __shared__ T s_chan[3][kMaxChan];
    if ((int)threadIdx.x < kMaxChan) {
        s_chan[0][threadIdx.x] = chan_pick(a.chan_dT, (int)threadIdx.x);
        s_chan[1][threadIdx.x] = chan_pick(g.chan_dph, (int)threadIdx.x);
        s_chan[2][threadIdx.x] = chan_pick(g.chan_dam, (int)threadIdx.x);
    }
    __syncthreads();
    // XCD-aware tile order, as in the forward kernel
    const int nwg = gridDim.x, b = blockIdx.x;
    const int q = nwg / kAdjXcds, rem = nwg % kAdjXcds, xcd = b % kAdjXcds, kk = b / kAdjXcds;
    const int L = xcd < rem ? xcd * (q + 1) + kk : rem * (q + 1) + (xcd - rem) * q + kk;
    const int tile_x = L % fg.tiles_x;
    const int tile_y = (L / fg.tiles_x) % fg.tiles_y;
    const int z0 = (L / (fg.tiles_x * fg.tiles_y)) * fg.zc;
    const int z1 = min(z0 + fg.zc, a.nz);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = tile_x * TX + tx, y = tile_y * TY + ty;
    const bool inxy = x < a.nx && y < a.ny;
    const unsigned nxy = (unsigned)a.nx * (unsigned)a.ny;
    const unsigned col = inxy ? (unsigned)x + (unsigned)a.nx * (unsigned)y : 0u;
    const int own = (tx + 1) + RW * (ty + 1);
    // ring cell of this thread (one-cell border, corners excluded)
    const bool ring = tid < 2 * (TX + TY);
    int rx = 0, ry = 0;
    if (tid < TY) { rx = -1; ry = tid; }
    else if (tid < 2 * TY) { rx = TX; ry = tid - TY; }
    else if (tid < 2 * TY + TX) { rx = tid - 2 * TY; ry = -1; }
    else if (ring) { rx = tid - 2 * TY - TX; ry = TY; }
    const int gxr = tile_x * TX + rx, gyr = tile_y * TY + ry;
    const bool ring_in = ring && gxr >= 0 && gxr < a.nx && gyr >= 0 && gyr < a.ny;
    const unsigned ring_col = ring_in ? (unsigned)gxr + (unsigned)a.nx * (unsigned)gyr : 0u;
    const int ring_slot = (rx + 1) + RW * (ry + 1);
    // bond entering the tile: x from (-1, tid) or y from (tid - TY, -1)
    const bool bnd = tid < TX + TY;
    const bool bnd_y = tid >= TY;
    const int bnd_lo = bnd_y ? (tid - TY + 1) : RW * (tid + 1);
    const int bnd_up = bnd_y ? bnd_lo + RW : bnd_lo + 1;
    const int bnd_i = bnd_y ? (tid - TY) : (TX + 1) * tid;
    const LatK<T> C = lat_consts(a.l);

    // Stage slab z in LDS: the own cell o and this thread's ring cell,
    // whose loads r were issued earlier.
    auto stage = [&](const AdjCell<T> &o, const AdjPre<T> &r) __attribute__((always_inline)) {
        if (inxy) {
            if (o.m) put_cell<T>(sm, own, o);
            sm.mat[own] = o.m;
        } else {
            sm.mat[own] = 0;
        }
        if (ring) {
            AdjCell<T> R{};
            if (ring_in) finish_adj(a, s_chan[0], r, R);
            if (R.m) put_cell<T>(sm, ring_slot, R);
            sm.mat[ring_slot] = R.m;
        }
    };

    AdjCell<T> A{}, B{};
    if (inxy && z0 < z1) load_cell(a, g, s_chan[0], col + (unsigned)z0 * nxy, A);
    AdjPre<T> rp{};
    if (ring_in && z0 < z1) issue_adj(a, g, ring_col + (unsigned)z0 * nxy, rp);
    // voxel-2 end of the bond entering the chunk from below
    T cin[kEnd];
    bool has_cin = false;
#pragma unroll
    for (int i = 0; i < kEnd; ++i) cin[i] = T(0);
    if (A.m && z0 > 0) {
        AdjCell<T> P{};
        load_cell(a, g, s_chan[0], col + (unsigned)(z0 - 1) * nxy, P);
        if (P.m) {
            T ea[kEnd];
            bond_ends<T, 2>(P, A, a.zeta_bond, C, ea, cin);
            has_cin = true;
        }
    }
    if (z0 < z1) stage(A, rp);

    // one slab: cur (slab z) is staged in LDS; slab z + 1 is staged once
    // every thread is past its bonds of slab z.  In FP32 the loads of slab
    // z + 1 (own cell and ring cell) are issued first and arrive during the
    // bond VJPs; FP64, whose registers are already full, issues them where
    // they are used.
    constexpr bool early = sizeof(T) == 4;
    auto slab = [&](AdjCell<T> &cur, AdjCell<T> &nxt, int z) __attribute__((always_inline)) {
        AdjPre<T> pn{};
        if constexpr (early) {
            if (inxy && z + 1 < a.nz) issue_adj(a, g, col + (unsigned)(z + 1) * nxy, pn);
            rp.m = 0;
            if (ring_in && z + 1 < z1) issue_adj(a, g, ring_col + (unsigned)(z + 1) * nxy, rp);
        }
        __syncthreads();

        // bonds entering the tile from the ring (only their inner end is kept)
        if (bnd && sm.mat[bnd_lo] && sm.mat[bnd_up]) {
            const AdjCell<T> Lc = get_cell<T>(sm, bnd_lo), U = get_cell<T>(sm, bnd_up);
            T ea[kEnd], eb[kEnd];
            if (bnd_y) {
                bond_ends<T, 1>(Lc, U, a.zeta_bond, C, ea, eb);
#pragma unroll
                for (int i = 0; i < kEnd; ++i) sm.ry[i][bnd_i] = eb[i];
            } else {
                bond_ends<T, 0>(Lc, U, a.zeta_bond, C, ea, eb);
#pragma unroll
                for (int i = 0; i < kEnd; ++i) sm.rx[i][bnd_i] = eb[i];
            }
        }
        T acc[kEnd];
#pragma unroll
        for (int i = 0; i < kEnd; ++i) acc[i] = T(0);
        if (cur.m && sm.mat[own + 1]) {
            const AdjCell<T> Bc = get_cell<T>(sm, own + 1);
            T ea[kEnd], eb[kEnd];
            bond_ends<T, 0>(cur, Bc, a.zeta_bond, C, ea, eb);
#pragma unroll
            for (int i = 0; i < kEnd; ++i) { acc[i] += ea[i]; sm.rx[i][(tx + 1) + (TX + 1) * ty] = eb[i]; }
        }
        if (cur.m && sm.mat[own + RW]) {
            const AdjCell<T> Bc = get_cell<T>(sm, own + RW);
            T ea[kEnd], eb[kEnd];
            bond_ends<T, 1>(cur, Bc, a.zeta_bond, C, ea, eb);
#pragma unroll
            for (int i = 0; i < kEnd; ++i) { acc[i] += ea[i]; sm.ry[i][tx + TX * (ty + 1)] = eb[i]; }
        }
        // neighbour materials for the gather, read before the slab's LDS is
        // restaged
        const bool n_mx = cur.m && sm.mat[own - 1] != 0;
        const bool n_my = cur.m && sm.mat[own - RW] != 0;
        nxt.m = 0;
        if (inxy && z + 1 < a.nz) {
            if constexpr (!early) issue_adj(a, g, col + (unsigned)(z + 1) * nxy, pn);
            finish_adj(a, s_chan[0], pn, nxt);
        }
        T cout[kEnd];
        const bool has_z = cur.m && nxt.m;
        if (has_z) {
            T ea[kEnd];
            bond_ends<T, 2>(cur, nxt, a.zeta_bond, C, ea, cout);
#pragma unroll
            for (int i = 0; i < kEnd; ++i) acc[i] += ea[i];
        }
        __syncthreads();

        // the bond ends stay in LDS until the next slab's first barrier; the
        // cells of slab z are no longer read
        if constexpr (!early) {
            rp.m = 0;
            if (ring_in && z + 1 < z1) issue_adj(a, g, ring_col + (unsigned)(z + 1) * nxy, rp);
        }
        if (z + 1 < z1) stage(nxt, rp);
        if (cur.m) {
            if (n_mx) {
#pragma unroll
                for (int i = 0; i < kEnd; ++i) acc[i] += sm.rx[i][tx + (TX + 1) * ty];
            }
            if (n_my) {
#pragma unroll
                for (int i = 0; i < kEnd; ++i) acc[i] += sm.ry[i][tx + TX * ty];
            }
            if (has_cin) {
#pragma unroll
                for (int i = 0; i < kEnd; ++i) acc[i] += cin[i];
            }
            finish_voxel(a, g, s_chan, col + (unsigned)z * nxy, cur.m, acc);
        }
        has_cin = has_z;
#pragma unroll
        for (int i = 0; i < kEnd; ++i) cin[i] = has_z ? cout[i] : T(0);
    };

    // one slab per trip (two per trip, without the copy, costs registers)
    for (int z = z0; z < z1; ++z) {
        slab(A, B, z);
        A = B;
    }
}

}  // namespace

template <typename T>
hipError_t launch_adjoint_fused(const StepArgs<T> &a, const AdjArgs<T> &g, hipStream_t s) {
    constexpr int TX = kAdjTX, TY = kAdjTY;
    AdjGrid fg;
    fg.tiles_x = (a.nx + TX - 1) / TX;
    fg.tiles_y = (a.ny + TY - 1) / TY;
    const long long cols = (long long)fg.tiles_x * fg.tiles_y;
    // two workgroups per CU in FP32 (255 VGPRs, 67 KB LDS), one in FP64
    fg.zc = balanced_zc(a.nz, cols, sizeof(T) == 4 ? 2 : 1);
    fg.chunks = (a.nz + fg.zc - 1) / fg.zc;
    k_adj_fused<T, TX, TY><<<(unsigned)(cols * fg.chunks), TX * TY, 0, s>>>(a, g, fg);
    return hipGetLastError();
}

template hipError_t launch_adjoint_fused<float>(const StepArgs<float> &, const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_fused<double>(const StepArgs<double> &, const AdjArgs<double> &, hipStream_t);

}  // namespace vx
