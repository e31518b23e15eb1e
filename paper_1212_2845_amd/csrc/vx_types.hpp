// Shared host/device types of the voxsim library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

// Per-voxel flag bits (one byte per cell).
enum : uint8_t {
    FLAG_FIXED = 1u << 0,    // immobile (fixed region)
    FLAG_STATIC = 1u << 1,   // floor static-friction state
    FLAG_SURFACE = 1u << 2,  // has an empty or out-of-grid face neighbour
    FLAG_FORCED = 1u << 3,   // has a constant external force
    FLAG_CAND = 1u << 4,     // has collision candidates (contact force buffer valid)
    FLAG_ACT = 1u << 5,      // own actuation amplitude/phase
    FLAG_CHAN = 1u << 6,     // follows a named actuation channel
};

// Named actuation channels per lattice.
constexpr int kMaxChan = 8;

// One value per channel, as scalar members: the step arguments are copied
// and modified inside kernels, and an array member would keep such a copy
// in private memory.
template <typename T>
struct Chan8 {
    T v0, v1, v2, v3, v4, v5, v6, v7;
};

template <typename T>
inline void chan_set(Chan8<T> &c, int k, T x) {
    switch (k) {
        case 0: c.v0 = x; break; case 1: c.v1 = x; break; case 2: c.v2 = x; break; case 3: c.v3 = x; break;
        case 4: c.v4 = x; break; case 5: c.v5 = x; break; case 6: c.v6 = x; break; default: c.v7 = x; break;
    }
}

// State words of one voxel, stored structure-of-arrays: word k of cell c is
// at base[k * stride + c].  Displacement from the rest position (not the
// absolute position) keeps FP32 increments representable.
enum : int {
    W_UX = 0, W_UY, W_UZ,
    W_QW, W_QX, W_QY, W_QZ,
    W_PX, W_PY, W_PZ,   // linear momentum
    W_LX, W_LY, W_LZ,   // angular momentum
    N_WORDS
};

// Per-material constants, precomputed on the host.
template <typename T>
struct MatConst {
    T m, inv_m;        // mass rho l^3 and its inverse
    T I, inv_I;        // rotational inertia m l^2 / 6 and its inverse
    T cg, cgr;         // ground damping coefficients 2 zeta_slow sqrt(m k), sqrt(I k_phi)
    T cfloor;          // floor normal damping 2 zeta_col sqrt(m k)
    T kv;              // voxel stiffness E l (floor penalty)
    T cte, mu_s, mu_d;
    T E;               // elastic modulus (contact stiffness)
    T gfac;            // 1 / (2 (1 + nu)): shear modulus per unit E
    T pad[3];
};

// Per-material-pair beam constants (Eq. 8-12) and bond damping (Eq. 34-35).
template <typename T>
struct PairConst {
    T a1, a2, b1, b2, b3;
    T ct, cr;          // 2 zeta_bond sqrt(m_min a1), 2 zeta_bond sqrt(I_min b3)
    T kc;              // contact stiffness E_c l
    T cc;              // contact damping 2 zeta_col sqrt(m_min kc)
    T pad;
};

// Small device-side scalars, one 256-byte block.
struct Scalars {
    unsigned err_flag;
    unsigned overflow;
    unsigned rebuild_flag;
    unsigned done;               // last-workgroup hand-off counter, 0 between launches
    unsigned long long vmax_bits;
    double macc;
    unsigned long long pair_count;
    unsigned long long rebuilds;
    double threshold;            // rebuild once 2 macc >= threshold (horizon - c_max)
    unsigned every;              // 1: rebuild before every step
};


// Everything a step kernel needs, passed by value.
template <typename T>
struct StepArgs {
    const T *s_in;
    T *s_out;
    long long stride;          // = ncell
    const uint8_t *mat;
    const uint8_t *flags;      // flags at t_n (read)
    uint8_t *flags_out;        // flags at t_n+1 (written for every filled voxel)
    const MatConst<T> *mats;
    const PairConst<T> *pairs;
    int n_mat;
    int nx, ny, nz;
    T l;
    T dt;
    T gravity;
    T origin_z;
    double origin[3];          // world position of the lower corner of cell 0
    T dT_global;               // temperature of voxels without own signal, at t_n
    double wt;                 // 2 pi f t_n
    T wt_red;                  // 2 pi f t_n reduced to [0, 2 pi)
    const T *act_amp;          // per cell, used where FLAG_ACT
    const T *act_phase;
    const uint8_t *chan;       // per cell, channel index, used where FLAG_CHAN
    Chan8<T> chan_dT;          // temperature of each channel at t_n
    const int *forced_cells;   // sorted
    const T *forced_F;         // n_forced x 3
    int n_forced;
    int floor_on;
    int track_vmax;
    const T *contact_F;        // 3 x ncell, valid where FLAG_CAND
    T *bonds;                  // split path: 3 axes x 9 words x ncell
    unsigned *err_flag;
    unsigned long long *vmax_bits;
    const T *E_cell;           // parameter mode: per-cell elastic modulus, or null
    const T *rho_cell;         // parameter mode: per-cell density (set whenever E_cell is)
    T *fm_out;                 // split gather: per-voxel bond force and moment sums (6 x ncell), or null
    T zeta_bond, zeta_slow, zeta_col;
};

}  // namespace vx
