// Fused step kernel: one launch per step, each voxel's state read from HBM
// once and written once.
//
// A workgroup owns a TX x TY column of cells and marches up a chunk of z
// slabs (2.5-D blocking).  For each slab the own cells and a one-cell ring
// around the tile are staged in LDS as kinematic quantities; every x- and
// y-bond touching the tile is evaluated once (bonds that enter the tile
// from the ring as well), its result kept in LDS, and the bond to the slab
// above is evaluated in registers with its voxel-2 half carried to the next
// slab.  The next slab's cells are loaded while the bonds are evaluated and
// staged in LDS between the bond pass and the update, so that neither the
// ring cells' loads nor their kinematics occupy registers during the
// update.  Each thread then sums its own voxel's at most six bond results in
// the fixed order -x, +x, -y, +y, -z, +z (no atomics) and integrates.  The
// per-bond and per-voxel arithmetic is the same device code as the split
// path; material and material-pair constants are staged in LDS once per
// workgroup.  In parameter mode (per-cell modulus and density) each cell's
// modulus and mass travel with its kinematics, the voxel and bond constants
// are derived from them as the split path does, and the per-voxel bond sums
// can be written out for the adjoint.
//
// Workgroups are numbered so that consecutive tiles land on the same XCD
// (the dispatcher deals workgroups round-robin over the 8 XCDs), keeping
// the ring loads of neighbouring tiles in one L2.
#include <type_traits>

#include "vx_device.hpp"
#include "vx_launch.hpp"

namespace vx {

namespace {

constexpr int kXcds = 8;
constexpr int kKin = 14;   // ux uy uz qw qx qy qz vx vy vz wx wy wz eps

// LDS of one workgroup: a slab of kinematics with its ring, and the x- and
// y-bond results (b[0] and b[1]), sized for NR ring cells and NBX / NBY
// bonds.  Both bond arrays have the larger length, so a bond whose axis is
// chosen per lane is stored through one address.  A bond result is the
// force on voxel 2 (words 0-2), the moment on voxel 2 (the last three words)
// and, with NW = 9, the moment on voxel 1 (words 3-5).  With NW = 6 the thread that evaluates a bond adds
// voxel 1's half to that voxel's sums at once: less LDS and fewer LDS
// accesses, at the price of six sums held in registers through the bond
// evaluations, which the FP32 palette kernel's register budget (three waves
// per SIMD) does not have room for.
template <typename T, int NR_, int NBX_, int NBY_, int NW_>
struct Smem {
    static constexpr int NR = NR_, NB = NBX_ > NBY_ ? NBX_ : NBY_, NW = NW_;
    T kin[kKin][NR];
    T b[2][NW][NB];
    uint8_t mat[NR];
};

// With parameter mode: each slot's modulus and mass as well.
template <typename T, int NR_, int NBX_, int NBY_, int NW_>
struct SmemP : Smem<T, NR_, NBX_, NBY_, NW_> {
    T pE[NR_], pM[NR_];
};

template <typename T, bool Param>
constexpr int tile_bond_words() { return sizeof(T) == 4 && !Param ? 9 : 6; }
template <typename T, int TX, int TY>
using TileSmem = Smem<T, (TX + 2) * (TY + 2), (TX + 1) * TY, TX * (TY + 1), tile_bond_words<T, false>()>;
template <typename T, int TX, int TY>
using TileSmemP = SmemP<T, (TX + 2) * (TY + 2), (TX + 1) * TY, TX * (TY + 1), tile_bond_words<T, true>()>;

struct FusedGrid {
    int tiles_x, tiles_y, chunks, zc;
};

template <typename T, int NR>
__device__ __forceinline__ void put_kin(T (*kin)[NR], int slot, const VoxKin<T> &k) {
    kin[0][slot] = k.ux; kin[1][slot] = k.uy; kin[2][slot] = k.uz;
    kin[3][slot] = k.qw; kin[4][slot] = k.qx; kin[5][slot] = k.qy; kin[6][slot] = k.qz;
    kin[7][slot] = k.vx; kin[8][slot] = k.vy; kin[9][slot] = k.vz;
    kin[10][slot] = k.wx; kin[11][slot] = k.wy; kin[12][slot] = k.wz;
    kin[13][slot] = k.eps;
}

template <typename T, int NR>
__device__ __forceinline__ VoxKin<T> get_kin(const T (*kin)[NR], int slot) {
    VoxKin<T> k;
    k.ux = kin[0][slot]; k.uy = kin[1][slot]; k.uz = kin[2][slot];
    k.qw = kin[3][slot]; k.qx = kin[4][slot]; k.qy = kin[5][slot]; k.qz = kin[6][slot];
    k.vx = kin[7][slot]; k.vy = kin[8][slot]; k.vz = kin[9][slot];
    k.wx = kin[10][slot]; k.wy = kin[11][slot]; k.wz = kin[12][slot];
    k.eps = kin[13][slot];
    return k;
}

template <typename T, int NB, int NW>
__device__ __forceinline__ void put_bond(T (*b)[NB], int i, const BondOut<T> &o) {
    b[0][i] = o.f2x; b[1][i] = o.f2y; b[2][i] = o.f2z;
    if constexpr (NW == 9) { b[3][i] = o.m1x; b[4][i] = o.m1y; b[5][i] = o.m1z; }
    b[NW - 3][i] = o.m2x; b[NW - 2][i] = o.m2y; b[NW - 1][i] = o.m2z;
}

// Voxel 1's half of a bond added to its force and moment sums.
template <typename T>
__device__ __forceinline__ void add_end1(const BondOut<T> &o, T &Fx, T &Fy, T &Fz, T &Mx, T &My, T &Mz) {
    Fx -= o.f2x; Fy -= o.f2y; Fz -= o.f2z;
    Mx += o.m1x; My += o.m1y; Mz += o.m1z;
}

// The state words of a cell through one buffer descriptor per state array.
// Word w lies w * stride * sizeof(T) bytes after word 0, an offset kept in a
// scalar register, so the 13 words of a cell share one 32-bit vector offset
// (c * sizeof(T)) and no per-word 64-bit address is formed or kept: with
// one pointer per word the two state arrays alone take 52 scalar
// registers, which the compiler spills into vector lanes and reads back
// before every load and store.  The descriptor spans the 13 words; its
// record count, the per-lane offset and the per-word offset are unsigned
// 32-bit byte counts, so the host runs this kernel only when that span is
// below 2^32 bytes.
constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit data format, gfx9 family

template <typename T>
struct StateBuf {
    __amdgpu_buffer_rsrc_t in, out;
    unsigned wb;   // bytes from one state word to the next
    // scalar offset of word w, as the unsigned 32-bit pattern the
    // instruction takes
    __device__ __forceinline__ int word(int w) const { return (int)((unsigned)w * wb); }
};

template <typename T>
__device__ __forceinline__ StateBuf<T> state_buf(const StepArgs<T> &a) {
    StateBuf<T> b;
    const unsigned bytes = (unsigned)(N_WORDS * a.stride * (long long)sizeof(T));
    b.in = __builtin_amdgcn_make_buffer_rsrc((void *)a.s_in, 0, (int)bytes, kRsrcWord3);
    b.out = __builtin_amdgcn_make_buffer_rsrc((void *)a.s_out, 0, (int)bytes, kRsrcWord3);
    b.wb = (unsigned)(a.stride * (long long)sizeof(T));
    return b;
}

template <typename T> __device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, int soff);
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, soff, 0));
}
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, soff, 0));
}
template <typename T> __device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, int soff, T v);
template <> __device__ __forceinline__ void buf_st<float>(__amdgpu_buffer_rsrc_t r, unsigned off, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, soff, 0);
}
template <> __device__ __forceinline__ void buf_st<double>(__amdgpu_buffer_rsrc_t r, unsigned off, int soff, double v) {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)off, soff, 0);
}

template <typename T>
__device__ __forceinline__ VoxRaw<T> sb_load(const StateBuf<T> &b, unsigned c) {
    const unsigned o = c * (unsigned)sizeof(T);
    VoxRaw<T> r;
    r.ux = buf_ld<T>(b.in, o, 0);           r.uy = buf_ld<T>(b.in, o, b.word(W_UY));
    r.uz = buf_ld<T>(b.in, o, b.word(W_UZ)); r.qw = buf_ld<T>(b.in, o, b.word(W_QW));
    r.qx = buf_ld<T>(b.in, o, b.word(W_QX)); r.qy = buf_ld<T>(b.in, o, b.word(W_QY));
    r.qz = buf_ld<T>(b.in, o, b.word(W_QZ)); r.px = buf_ld<T>(b.in, o, b.word(W_PX));
    r.py = buf_ld<T>(b.in, o, b.word(W_PY)); r.pz = buf_ld<T>(b.in, o, b.word(W_PZ));
    r.lx = buf_ld<T>(b.in, o, b.word(W_LX)); r.ly = buf_ld<T>(b.in, o, b.word(W_LY));
    r.lz = buf_ld<T>(b.in, o, b.word(W_LZ));
    return r;
}

template <typename T>
__device__ __forceinline__ void sb_store(const StateBuf<T> &b, unsigned c, const VoxRaw<T> &v) {
    const unsigned o = c * (unsigned)sizeof(T);
    buf_st<T>(b.out, o, 0, v.ux);           buf_st<T>(b.out, o, b.word(W_UY), v.uy);
    buf_st<T>(b.out, o, b.word(W_UZ), v.uz); buf_st<T>(b.out, o, b.word(W_QW), v.qw);
    buf_st<T>(b.out, o, b.word(W_QX), v.qx); buf_st<T>(b.out, o, b.word(W_QY), v.qy);
    buf_st<T>(b.out, o, b.word(W_QZ), v.qz); buf_st<T>(b.out, o, b.word(W_PX), v.px);
    buf_st<T>(b.out, o, b.word(W_PY), v.py); buf_st<T>(b.out, o, b.word(W_PZ), v.pz);
    buf_st<T>(b.out, o, b.word(W_LX), v.lx); buf_st<T>(b.out, o, b.word(W_LY), v.ly);
    buf_st<T>(b.out, o, b.word(W_LZ), v.lz);
}

// Own voxel of one slab: material, flags, strain, raw state, kinematics.
template <typename T>
struct Own {
    uint8_t m, fl;
    T eps;
    VoxRaw<T> r;
    VoxKin<T> k;
};

// Raw words of one cell in flight: material, flags and all state words,
// loaded without waiting on any of them (also for an empty cell, whose
// state words exist and are ignored), so that a prefetch one slab ahead
// costs no stall until the values are used.
template <typename T>
struct Pre {
    uint8_t m, fl;
    VoxRaw<T> r;
};

// The same with the cell's modulus and density (parameter mode).
template <typename T>
struct OwnP : Own<T> {
    T E, rho;
};
template <typename T>
struct PreP : Pre<T> {
    T E, rho;
};
template <bool Param, typename T>
using OwnT = typename std::conditional<Param, OwnP<T>, Own<T>>::type;
template <bool Param, typename T>
using PreT = typename std::conditional<Param, PreP<T>, Pre<T>>::type;

// Per-workgroup copies of the material and material-pair tables and of the
// actuation channels' temperatures at t_n.
template <typename T>
struct Tables {
    const MatConst<T> *mat;   // n_mat entries
    const T *pair;            // n_mat^2 x 4: a1, a2, ct, -
    const T *chan;            // kMaxChan entries
    int n_mat;
    __device__ __forceinline__ BondK<T> bond(int m1, int m2) const {
        const T *p = pair + 4 * (m1 * n_mat + m2);
        BondK<T> k;
        k.a1 = p[0]; k.a2 = p[1]; k.ct = p[2];
        return k;
    }
};

// voxel_strain with the channel temperatures read from the workgroup's
// table (the step arguments' copies are not kept in registers); lattices
// without channel voxels take the kernels built without the channel test.
template <bool Chan, typename T>
__device__ __forceinline__ T strain_tb(const StepArgs<T> &a, const Tables<T> &tb, unsigned c, uint8_t fl, T cte) {
    if constexpr (Chan) {
        if (fl & FLAG_CHAN) return cte * tb.chan[ldc(a.chan, c)];
    }
    return signal_strain(a, c, fl, cte);
}

// f(constants of the voxel of o, an Own or a Pre): the workgroup's table
// entry of its material, or in parameter mode the entry with the cell's own
// modulus and density (as mat_at computes them).
template <bool Param, typename T, typename O, typename F>
__device__ __forceinline__ void with_mc(const StepArgs<T> &a, const Tables<T> &tb, const O &o, const F &f) {
    if constexpr (Param) f(mat_with(tb.mat[o.m], o.E, o.rho, a.l, a.zeta_slow, a.zeta_col));
    else f(tb.mat[o.m]);
}

template <bool Chan, bool Param, typename T>
__device__ __forceinline__ void load_own(const StepArgs<T> &a, const StateBuf<T> &sb, const Tables<T> &tb,
                                         unsigned c, OwnT<Param, T> &o) {
    o.m = ldc(a.mat, c);
    if (o.m) {
        o.fl = ldc(a.flags, c);
        o.r = sb_load(sb, c);
        if constexpr (Param) { o.E = ldc(a.E_cell, c); o.rho = ldc(a.rho_cell, c); }
        with_mc<Param>(a, tb, o, [&](const MatConst<T> &mc) __attribute__((always_inline)) {
            o.eps = strain_tb<Chan>(a, tb, c, o.fl, mc.cte);
            o.k = kin_of(o.r, mc, o.eps);
        });
    }
}


template <bool Param, typename T>
__device__ __forceinline__ void issue_pre(const StepArgs<T> &a, const StateBuf<T> &sb, unsigned c,
                                          PreT<Param, T> &p) {
    p.m = ldc(a.mat, c);
    p.fl = ldc(a.flags, c);
    p.r = sb_load(sb, c);
    if constexpr (Param) { p.E = ldc(a.E_cell, c); p.rho = ldc(a.rho_cell, c); }
}

// Strain and kinematics of a prefetched cell.
template <bool Chan, bool Param, typename T>
__device__ __forceinline__ void finish_pre(const StepArgs<T> &a, const Tables<T> &tb, unsigned c,
                                           const PreT<Param, T> &p, OwnT<Param, T> &o) {
    o.m = p.m;
    if (p.m) {
        o.fl = p.fl;
        o.r = p.r;
        if constexpr (Param) { o.E = p.E; o.rho = p.rho; }
        with_mc<Param>(a, tb, p, [&](const MatConst<T> &mc) __attribute__((always_inline)) {
            o.eps = strain_tb<Chan>(a, tb, c, p.fl, mc.cte);
            o.k = kin_of(p.r, mc, o.eps);
        });
    }
}

// Load the material tables into LDS (all threads of the workgroup; the
// caller synchronises before use).
template <typename T>
__device__ __forceinline__ Tables<T> stage_tables(const StepArgs<T> &a, unsigned char *dyn, int nthreads) {
    Tables<T> tb;
    tb.n_mat = a.n_mat;
    MatConst<T> *smat = (MatConst<T> *)dyn;
    T *spair = (T *)(dyn + ((a.n_mat * sizeof(MatConst<T>) + 15) & ~(size_t)15));
    const T *gm = (const T *)a.mats;
    T *sm_ = (T *)smat;
    const int nmw = a.n_mat * (int)(sizeof(MatConst<T>) / sizeof(T));
    for (int i = threadIdx.x; i < nmw; i += nthreads) sm_[i] = gm[i];
    const int np = a.n_mat * a.n_mat;
    for (int i = threadIdx.x; i < np; i += nthreads) {
        spair[4 * i] = a.pairs[i].a1;
        spair[4 * i + 1] = a.pairs[i].a2;
        spair[4 * i + 2] = a.pairs[i].ct;
        spair[4 * i + 3] = T(0);
    }
    T *schan = spair + 4 * np;
    if ((int)threadIdx.x < kMaxChan) schan[threadIdx.x] = chan_pick(a.chan_dT, (int)threadIdx.x);
    tb.mat = smat;
    tb.pair = spair;
    tb.chan = schan;
    return tb;
}

template <typename T>
__host__ __device__ inline size_t tables_bytes(int n_mat) {
    return ((n_mat * sizeof(MatConst<T>) + 15) & ~(size_t)15) + (size_t)n_mat * n_mat * 4 * sizeof(T) +
           kMaxChan * sizeof(T);
}

// One column of cells: the TX x TY tile (tile_x, tile_y) of lattice a,
// marched over slabs [z0, z1).  Called by every thread of the workgroup
// (threads beyond TX * TY only help with the ring and the barriers).  TX and
// TY may be compile-time constants (fused kernel) or runtime values within
// the LDS sizes of S (batched kernel).
template <bool Chan, bool Param, typename T, typename S>
__device__ __forceinline__ void march(const StepArgs<T> &a, S &sm, const Tables<T> &tb, const LatK<T> &C,
                                      const int TX, const int TY, int tile_x, int tile_y, int z0, int z1,
                                      T &vmax) {
    constexpr int NR = S::NR, NB = S::NB, NW = S::NW;
    constexpr bool kEnd1Regs = NW == 6;
    const int RW = TX + 2;
    const int tid = threadIdx.x;
    const bool lane_in = tid < TX * TY;
    const int tx = lane_in ? tid % TX : 0, ty = lane_in ? tid / TX : 0;
    const int x = tile_x * TX + tx, y = tile_y * TY + ty;
    const bool inxy = lane_in && x < a.nx && y < a.ny;
    const unsigned nxy = (unsigned)a.nx * (unsigned)a.ny;
    const unsigned col = inxy ? (unsigned)x + (unsigned)a.nx * (unsigned)y : 0u;
    const int own = (tx + 1) + RW * (ty + 1);
    const StateBuf<T> sb = state_buf(a);
    // mass of a voxel of density rho (as mat_with), and the constants of the
    // bond between materials m1, m2 with moduli E1, E2 and masses M1, M2
    auto mass = [&](T rho) __attribute__((always_inline)) { return rho * a.l * a.l * a.l; };
    auto bond_kc = [&](uint8_t m1, uint8_t m2, T E1, T E2, T M1, T M2) __attribute__((always_inline)) {
        if constexpr (Param)
            return bond_k_from_E(E1, E2, tb.mat[m1].gfac, tb.mat[m2].gfac, M1 < M2 ? M1 : M2, a.zeta_bond, C);
        else
            return tb.bond(m1, m2);
    };
    // the same between two cells held in registers
    auto bond_oo = [&](const OwnT<Param, T> &p, const OwnT<Param, T> &q) __attribute__((always_inline)) {
        if constexpr (Param) return bond_kc(p.m, q.m, p.E, q.E, mass(p.rho), mass(q.rho));
        else return tb.bond(p.m, q.m);
    };

    // ring cell of this thread (one-cell border of the tile, corners excluded)
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
    // boundary bond entering the tile: x from (-1, tid) or y from (tid - TY, -1)
    const bool bnd = tid < TX + TY;
    const bool bnd_y = tid >= TY;
    const int bnd_lo = bnd_y ? (tid - TY + 1) : RW * (tid + 1);
    const int bnd_up = bnd_y ? bnd_lo + RW : bnd_lo + 1;
    const int bnd_i = bnd_y ? (tid - TY) : (TX + 1) * tid;

    // Stage slab z in LDS: kinematics and material of the own cell o and of
    // this thread's ring cell, whose loads r were issued earlier.
    auto stage = [&](const OwnT<Param, T> &o, const PreT<Param, T> &r, int z) __attribute__((always_inline)) {
        if (lane_in) {
            if (o.m) {
                put_kin<T, NR>(sm.kin, own, o.k);
                if constexpr (Param) { sm.pE[own] = o.E; sm.pM[own] = mass(o.rho); }
            }
            sm.mat[own] = o.m;
        }
        if (ring) {
            uint8_t mr = 0;
            if (ring_in) {
                OwnT<Param, T> R{};
                finish_pre<Chan, Param>(a, tb, ring_col + (unsigned)z * nxy, r, R);
                mr = R.m;
                if (mr) {
                    put_kin<T, NR>(sm.kin, ring_slot, R.k);
                    if constexpr (Param) { sm.pE[ring_slot] = R.E; sm.pM[ring_slot] = mass(R.rho); }
                }
            }
            sm.mat[ring_slot] = mr;
        }
    };

    OwnT<Param, T> A{}, B{};
    if (inxy && z0 < z1) load_own<Chan, Param>(a, sb, tb, col + (unsigned)z0 * nxy, A);
    PreT<Param, T> rp{};
    if (ring_in && z0 < z1) issue_pre<Param>(a, sb, ring_col + (unsigned)z0 * nxy, rp);

    // bond from the slab below the chunk: only its voxel-2 half is needed
    bool has_carry = false;
    T cFx = T(0), cFy = T(0), cFz = T(0), cMx = T(0), cMy = T(0), cMz = T(0);
    if (A.m && z0 > 0) {
        OwnT<Param, T> P{};
        load_own<Chan, Param>(a, sb, tb, col + (unsigned)(z0 - 1) * nxy, P);
        if (P.m) {
            const Rot<T> Rp = rot_of(P.k.qw, P.k.qx, P.k.qy, P.k.qz);
            const BondOut<T> o =
                bond_eval<T, 2>(P.k, Rp, A.k, bond_oo(P, A), C);
            cFx = o.f2x; cFy = o.f2y; cFz = o.f2z; cMx = o.m2x; cMy = o.m2y; cMz = o.m2z;
            has_carry = true;
        }
    }
    if (z0 < z1) stage(A, rp, z0);

    // one slab: cur holds slab z, already staged in LDS; nxt receives slab
    // z + 1, whose loads (own cell and ring cell) are issued at the start so
    // that they arrive during the bond evaluations, and which is staged in
    // LDS once every thread is past its bonds of slab z
    auto slab = [&](OwnT<Param, T> &cur, OwnT<Param, T> &nxt, int z) __attribute__((always_inline)) {
        PreT<Param, T> pn{};
        if (inxy && z + 1 < a.nz) issue_pre<Param>(a, sb, col + (unsigned)(z + 1) * nxy, pn);
        rp.m = 0;
        if (ring_in && z + 1 < z1) issue_pre<Param>(a, sb, ring_col + (unsigned)(z + 1) * nxy, rp);
        __syncthreads();

        // bonds entering the tile from the ring: x from (-1, tid), y from
        // (tid - TY, -1)
        if (bnd) {
            const uint8_t ml = sm.mat[bnd_lo], mu = sm.mat[bnd_up];
            if (ml && mu) {
                const VoxKin<T> kl = get_kin<T, NR>(sm.kin, bnd_lo), ku = get_kin<T, NR>(sm.kin, bnd_up);
                const Rot<T> Rl = rot_of(kl.qw, kl.qx, kl.qy, kl.qz);
                T El = T(0), Eu = T(0), Ml = T(0), Mu = T(0);
                if constexpr (Param) { El = sm.pE[bnd_lo]; Eu = sm.pE[bnd_up]; Ml = sm.pM[bnd_lo]; Mu = sm.pM[bnd_up]; }
                const BondOut<T> o = bond_eval_xy(kl, Rl, ku, bond_kc(ml, mu, El, Eu, Ml, Mu), C, bnd_y);
                put_bond<T, NB, NW>(sm.b[bnd_y ? 1 : 0], bnd_i, o);
            }
        }
        const Rot<T> Rc = rot_of(cur.k.qw, cur.k.qx, cur.k.qy, cur.k.qz);
        // bond constants with the neighbour in LDS slot sl
        auto kn = [&](uint8_t mu, int sl) __attribute__((always_inline)) {
            if constexpr (Param) return bond_kc(cur.m, mu, cur.E, sm.pE[sl], mass(cur.rho), sm.pM[sl]);
            else return tb.bond(cur.m, mu);
        };
        // the voxel's force and moment sums; with kEnd1Regs they start from
        // the bond below (carried from the previous slab or evaluated at the
        // chunk's start) and take the voxel-1 half of the +x, +y and +z bonds
        // as these are evaluated
        T Fx = T(0), Fy = T(0), Fz = T(0), Mx = T(0), My = T(0), Mz = T(0);
        if constexpr (kEnd1Regs) { Fx = cFx; Fy = cFy; Fz = cFz; Mx = cMx; My = cMy; Mz = cMz; }
        {
            const uint8_t mu = lane_in ? sm.mat[own + 1] : 0;
            if (cur.m && mu) {
                const VoxKin<T> ku = get_kin<T, NR>(sm.kin, own + 1);
                const BondOut<T> o = bond_eval<T, 0>(cur.k, Rc, ku, kn(mu, own + 1), C);
                put_bond<T, NB, NW>(sm.b[0], (tx + 1) + (TX + 1) * ty, o);
                if constexpr (kEnd1Regs) add_end1(o, Fx, Fy, Fz, Mx, My, Mz);
            }
        }
        {
            const uint8_t mu = lane_in ? sm.mat[own + RW] : 0;
            if (cur.m && mu) {
                const VoxKin<T> ku = get_kin<T, NR>(sm.kin, own + RW);
                const BondOut<T> o = bond_eval<T, 1>(cur.k, Rc, ku, kn(mu, own + RW), C);
                put_bond<T, NB, NW>(sm.b[1], tx + TX * (ty + 1), o);
                if constexpr (kEnd1Regs) add_end1(o, Fx, Fy, Fz, Mx, My, Mz);
            }
        }
        // neighbour materials for the gather, read before the slab's LDS is
        // restaged
        bool n_mx = false, n_px = false, n_my = false, n_py = false;
        if (lane_in) {
            n_mx = sm.mat[own - 1] != 0; n_px = sm.mat[own + 1] != 0;
            n_my = sm.mat[own - RW] != 0; n_py = sm.mat[own + RW] != 0;
        }
        finish_pre<Chan, Param>(a, tb, col + (unsigned)(z + 1) * nxy, pn, nxt);
        const bool has_zb = cur.m && nxt.m;
        BondOut<T> oz{};
        if (has_zb)
            oz = bond_eval<T, 2>(cur.k, Rc, nxt.k, bond_oo(cur, nxt), C);
        if constexpr (kEnd1Regs) {
            if (has_zb) add_end1(oz, Fx, Fy, Fz, Mx, My, Mz);
            cFx = oz.f2x; cFy = oz.f2y; cFz = oz.f2z; cMx = oz.m2x; cMy = oz.m2y; cMz = oz.m2z;
        }
        __syncthreads();

        // the bond results stay in LDS until the next slab's first barrier;
        // the kinematics of slab z are no longer read
        if (z + 1 < z1) stage(nxt, rp, z + 1);
        if (cur.m) {
            if (n_mx) {
                const int i = tx + (TX + 1) * ty;
                Fx += sm.b[0][0][i]; Fy += sm.b[0][1][i]; Fz += sm.b[0][2][i];
                Mx += sm.b[0][NW - 3][i]; My += sm.b[0][NW - 2][i]; Mz += sm.b[0][NW - 1][i];
            }
            if constexpr (!kEnd1Regs) {
                if (n_px) {
                    const int i = (tx + 1) + (TX + 1) * ty;
                    Fx -= sm.b[0][0][i]; Fy -= sm.b[0][1][i]; Fz -= sm.b[0][2][i];
                    Mx += sm.b[0][3][i]; My += sm.b[0][4][i]; Mz += sm.b[0][5][i];
                }
            }
            if (n_my) {
                const int i = tx + TX * ty;
                Fx += sm.b[1][0][i]; Fy += sm.b[1][1][i]; Fz += sm.b[1][2][i];
                Mx += sm.b[1][NW - 3][i]; My += sm.b[1][NW - 2][i]; Mz += sm.b[1][NW - 1][i];
            }
            if constexpr (!kEnd1Regs) {
                if (n_py) {
                    const int i = tx + TX * (ty + 1);
                    Fx -= sm.b[1][0][i]; Fy -= sm.b[1][1][i]; Fz -= sm.b[1][2][i];
                    Mx += sm.b[1][3][i]; My += sm.b[1][4][i]; Mz += sm.b[1][5][i];
                }
                if (has_carry) {
                    Fx += cFx; Fy += cFy; Fz += cFz;
                    Mx += cMx; My += cMy; Mz += cMz;
                }
                if (has_zb) {
                    Fx -= oz.f2x; Fy -= oz.f2y; Fz -= oz.f2z;
                    Mx += oz.m1x; My += oz.m1y; Mz += oz.m1z;
                }
            }
            if constexpr (Param) {
                if (a.fm_out) {
                    const long long st = a.stride, c = col + (unsigned)z * nxy;
                    a.fm_out[0 * st + c] = Fx; a.fm_out[1 * st + c] = Fy; a.fm_out[2 * st + c] = Fz;
                    a.fm_out[3 * st + c] = Mx; a.fm_out[4 * st + c] = My; a.fm_out[5 * st + c] = Mz;
                }
            }
            with_mc<Param>(a, tb, cur, [&](const MatConst<T> &mc) __attribute__((always_inline)) {
                voxel_update(a, col + (unsigned)z * nxy, cur.fl, mc, cur.eps, cur.r, Fx, Fy, Fz, Mx, My, Mz, &vmax,
                             [&](unsigned c, const VoxRaw<T> &o) { sb_store(sb, c, o); });
            });
        }
        if constexpr (!kEnd1Regs) {
            has_carry = has_zb;
            cFx = oz.f2x; cFy = oz.f2y; cFz = oz.f2z; cMx = oz.m2x; cMy = oz.m2y; cMz = oz.m2z;
        }
    };

    // two slabs per trip so that the roles of A and B alternate without copies
    for (int z = z0; z < z1; z += 2) {
        slab(A, B, z);
        if (z + 1 < z1) slab(B, A, z + 1);
    }
}

// FP32 is held to 168 VGPRs, so that three workgroups share a CU (three
// waves per SIMD; two loop-invariant values go to scratch); in parameter
// mode, which derives every bond's constants from the two moduli and
// masses, it needs about 200 and runs two (fused_wg_per_cu); FP64 needs
// more than 256 and runs one wave per SIMD.
template <typename T, int TX, int TY, bool Chan, bool Param>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(fused_wg_per_cu(sizeof(T), Param))))
k_fused(StepArgs<T> a, FusedGrid g) {
    static_assert(2 * (TX + TY) <= TX * TY, "ring must fit one cell per thread");
    __shared__ typename std::conditional<Param, TileSmemP<T, TX, TY>, TileSmem<T, TX, TY>>::type sm;
    extern __shared__ __align__(16) unsigned char dyn[];
    const Tables<T> tb = stage_tables(a, dyn, TX * TY);
    const LatK<T> C = lat_consts(a.l);

    // XCD-aware tile order (bijective for any grid size)
    const int nwg = gridDim.x, b = blockIdx.x;
    const int q = nwg / kXcds, rem = nwg % kXcds, xcd = b % kXcds, kk = b / kXcds;
    const int L = xcd < rem ? xcd * (q + 1) + kk : rem * (q + 1) + (xcd - rem) * q + kk;
    const int tile_x = L % g.tiles_x;
    const int tile_y = (L / g.tiles_x) % g.tiles_y;
    const int chunk = L / (g.tiles_x * g.tiles_y);
    const int z0 = chunk * g.zc;
    const int z1 = min(z0 + g.zc, a.nz);
    __syncthreads();

    T vmax = T(0);
    march<Chan, Param>(a, sm, tb, C, TX, TY, tile_x, tile_y, z0, z1, vmax);
    if (a.track_vmax) wave_vmax(a.vmax_bits, vmax);
}

// Largest runtime tile of the batched kernel: TX, TY <= 64, TX * TY <= 256,
// so (TX + 2)(TY + 2) <= 396 ring slots and (TX + 1) TY, TX (TY + 1) <= 320.
constexpr int kBatchThreads = 256;
using BatchSmemF = Smem<float, 396, 320, 320, 6>;
using BatchSmemD = Smem<double, 396, 320, 320, 6>;
template <typename T> struct BatchSmemOf;
template <> struct BatchSmemOf<float> { using type = BatchSmemF; };
template <> struct BatchSmemOf<double> { using type = BatchSmemD; };

// Batched persistent step: each workgroup owns a list of whole objects and
// runs every step of the launch for all of them, with only workgroup
// barriers between steps (objects are independent, so no grid-wide sync).
// Each object's x-y extent is covered by runtime TX x TY tiles; per-object
// timestep and time.
template <typename T>
__global__ void __launch_bounds__(kBatchThreads) k_batch(BatchArgs<T> b) {
    __shared__ typename BatchSmemOf<T>::type sm;
    extern __shared__ __align__(16) unsigned char dyn[];
    const Tables<T> tb = stage_tables(b.base, dyn, kBatchThreads);
    const LatK<T> C = lat_consts(b.base.l);
    __syncthreads();
    const int o0 = b.wg_start[blockIdx.x], o1 = b.wg_start[blockIdx.x + 1];
    T vmax = T(0);
    for (int k = 0; k < b.steps; ++k) {
        const int p = (b.cur0 + k) & 1;
        const long long n = b.step0 + k;
        for (int oi = o0; oi < o1; ++oi) {
            const BatchObj<T> ob = b.objs[b.wg_objs[oi]];
            StepArgs<T> a = b.base;
            a.s_in = b.state[p] + ob.off;
            a.s_out = b.state[1 - p] + ob.off;
            a.mat = b.base.mat + ob.off;
            a.flags = b.flags[p] + ob.off;
            a.flags_out = b.flags[1 - p] + ob.off;
            if (a.contact_F) a.contact_F = b.base.contact_F + ob.off;
            a.nx = ob.nx; a.ny = ob.ny; a.nz = ob.nz;
            a.dt = ob.dt;
            a.origin_z = ob.origin_z;
            const double wt = 6.283185307179586 * b.temp_freq * ((double)n * (double)ob.dt);
            a.dT_global = (T)(b.temp_amp * sin(wt + b.temp_phase));
            a.wt = wt;
            a.wt_red = (T)fmod(wt, 6.283185307179586);
            const int tiles_x = (ob.nx + ob.tx - 1) / ob.tx, tiles_y = (ob.ny + ob.ty - 1) / ob.ty;
            for (int ty = 0; ty < tiles_y; ++ty)
                for (int tx = 0; tx < tiles_x; ++tx)
                    march<false, false>(a, sm, tb, C, ob.tx, ob.ty, tx, ty, 0, ob.nz, vmax);
        }
        // this step's writes are the next step's reads (same workgroup)
        __syncthreads();
    }
    if (b.base.track_vmax) wave_vmax(b.base.vmax_bits, vmax);
}

template <typename T, int TX, int TY>
hipError_t launch_tiles(const StepArgs<T> &a, int zc, bool chan, hipStream_t s) {
    FusedGrid g;
    g.tiles_x = (a.nx + TX - 1) / TX;
    g.tiles_y = (a.ny + TY - 1) / TY;
    const long long cols = (long long)g.tiles_x * g.tiles_y;
    if (zc <= 0) zc = balanced_zc(a.nz, cols, fused_wg_per_cu((int)sizeof(T), a.E_cell != nullptr));
    zc = zc > a.nz ? a.nz : zc;
    g.zc = zc;
    g.chunks = (a.nz + zc - 1) / zc;
    const long long nwg = cols * g.chunks;
    // parameter mode takes the variant with the channel test (a voxel without
    // a channel follows the global signal there too)
    if (a.E_cell)
        k_fused<T, TX, TY, true, true><<<(unsigned)nwg, TX * TY, tables_bytes<T>(a.n_mat), s>>>(a, g);
    else if (chan)
        k_fused<T, TX, TY, true, false><<<(unsigned)nwg, TX * TY, tables_bytes<T>(a.n_mat), s>>>(a, g);
    else
        k_fused<T, TX, TY, false, false><<<(unsigned)nwg, TX * TY, tables_bytes<T>(a.n_mat), s>>>(a, g);
    return hipGetLastError();
}

}  // namespace

int device_cus() {
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return 256;
    }
    if (cache[dev] > 0) return cache[dev];
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    cache[dev] = n;
    return n;
}

int balanced_zc(int nz, long long cols, int wg_per_cu) {
    const long long slots = (long long)device_cus() * wg_per_cu;
    // a large lattice fills the chip many times over whatever the chunk:
    // chunks of nz * cols / 4096 slabs (at least 4, so that the extra slab
    // below each chunk stays cheap), which keep the tail of the launch short
    if ((long long)nz * cols >= 32 * slots) {
        long long zc = ((long long)nz * cols + 4095) / 4096;
        if (zc < 4) zc = 4;
        return (int)(zc > nz ? nz : zc);
    }
    // otherwise the number of rounds of resident workgroups decides: the
    // chunk minimising rounds x (zc + 1) slab passes (the extra one for the
    // chunk's lower bond), the smaller chunk on a tie
    int best = nz;
    long long best_cost = -1;
    for (int zc = 1; zc <= nz; ++zc) {
        const long long chunks = (nz + zc - 1) / zc;
        const long long rounds = (cols * chunks + slots - 1) / slots;
        const long long cost = rounds * (zc + 1);
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = zc; }
    }
    return best;
}

const FusedShape kFusedShapes[kNumFusedShapes] = {{32, 8}, {64, 4}, {16, 16}, {50, 5}, {20, 12}};

template <typename T>
hipError_t launch_fused_step(const StepArgs<T> &a, const FusedCfg &cfg, hipStream_t s) {
    switch (cfg.shape) {
        case 1: return launch_tiles<T, 64, 4>(a, cfg.zc, cfg.chan != 0, s);
        case 2: return launch_tiles<T, 16, 16>(a, cfg.zc, cfg.chan != 0, s);
        case 3: return launch_tiles<T, 50, 5>(a, cfg.zc, cfg.chan != 0, s);
        case 4: return launch_tiles<T, 20, 12>(a, cfg.zc, cfg.chan != 0, s);
        default: return launch_tiles<T, 32, 8>(a, cfg.zc, cfg.chan != 0, s);
    }
}

template <typename T>
hipError_t launch_batch(const BatchArgs<T> &b, int n_wg, hipStream_t s) {
    k_batch<T><<<(unsigned)n_wg, kBatchThreads, tables_bytes<T>(b.base.n_mat), s>>>(b);
    return hipGetLastError();
}

template hipError_t launch_batch<float>(const BatchArgs<float> &, int, hipStream_t);
template hipError_t launch_batch<double>(const BatchArgs<double> &, int, hipStream_t);
template hipError_t launch_fused_step<float>(const StepArgs<float> &, const FusedCfg &, hipStream_t);
template hipError_t launch_fused_step<double>(const StepArgs<double> &, const FusedCfg &, hipStream_t);

}  // namespace vx
