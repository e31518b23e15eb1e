// Kernel launchers shared between the host API and the kernel files.
#pragma once

#include "vx_types.hpp"

namespace vx {

// Split path: three per-axis bond kernels then the gather/integrate kernel.
template <typename T>
hipError_t launch_split_step(const StepArgs<T> &a, hipStream_t s);

// Reverse of one split step (parameter mode, no self-collision).  a holds
// the forward step's arguments at t_n (s_in = x_n, flags at t_n, E_cell);
// the adjoint buffers are laid out like the state (word k of cell c at
// k * stride + c).
template <typename T>
struct AdjArgs {
    const T *fm;            // bond force and moment sums at x_n, 6 words
    const T *lam_in;        // adjoint of x_n+1, 13 words
    T *lam_out;             // adjoint of x_n, 13 words
    T *gfm;                 // adjoint of the bond sums, 6 words
    T *gloc;                // update's adjoints of the strain, modulus and mass, 3 words
    double *g_E, *g_rho, *g_phase, *g_amp;   // accumulated over the reverse steps
    Chan8<T> chan_dph;      // each channel's temperature derivative w.r.t. its phase, at t_n
    Chan8<T> chan_dam;      // and w.r.t. its amplitude
};

struct CollideArgs;
// One reverse step: the update's reverse per voxel, the contact forces'
// reverse when c is given (self-collision), then the bonds' reverse.
template <typename T>
hipError_t launch_adjoint_step(const StepArgs<T> &a, const AdjArgs<T> &g, const CollideArgs *c, hipStream_t s);
// Bond pass and gather of the reverse step in one LDS-tiled launch (after
// the per-voxel update VJP); no per-bond records.
template <typename T>
hipError_t launch_adjoint_fused(const StepArgs<T> &a, const AdjArgs<T> &g, hipStream_t s);

// Energies and momenta of the current state (a.s_in): kEnergyWords FP64
// partial sums per workgroup of energy_blocks(ncell) workgroups.
constexpr int kEnergyWords = 10;   // KE, U_elastic, U_gravity, U_floor, P (3), L (3)
int energy_blocks(long long ncell);
template <typename T>
hipError_t launch_energy(const StepArgs<T> &a, double *partials, hipStream_t s);
// Fixed-order device sum of launch_energy's partials into out[0..kEnergyWords).
hipError_t launch_energy_sum(const double *partials, long long ncell, double *out, hipStream_t s);
template <typename T>
hipError_t launch_probe(const T *state, long long stride, long long ncell, const int32_t *cells, int n, int word,
                        T *out, hipStream_t s);

// Fused path: one LDS-tiled kernel per step.  cfg.shape indexes
// kFusedShapes (tile TX x TY); cfg.zc is the z chunk per workgroup (0 picks
// balanced_zc for the kernel's occupancy, fused_wg_per_cu).
struct FusedShape {
    int tx, ty;
};
constexpr int kNumFusedShapes = 5;
extern const FusedShape kFusedShapes[kNumFusedShapes];
struct FusedCfg {
    int shape;
    int zc;
    int chan;   // 1: some voxel follows a named channel
};
// Compute units of the current device (256 if it cannot be queried).
int device_cus();
// Default z chunk of a column-marching kernel with cols tile columns and
// wg_per_cu resident workgroups per CU.
int balanced_zc(int nz, long long cols, int wg_per_cu);
// Resident workgroups per CU of the fused step kernel (register-bound), by
// element size and parameter mode.
constexpr int fused_wg_per_cu(int tsize, bool param) { return tsize == 4 ? (param ? 2 : 3) : 1; }
// Linear statics (matrix-free conjugate gradients): the lattice and the
// per-cell moduli of the direct-stiffness operator.
struct StaticArgs {
    int nx, ny, nz;
    long long n;                 // cells
    double l;
    const uint8_t *mat;          // material per cell (0 = empty)
    const uint8_t *fixed;        // 1 = clamped
    const double *E, *G;         // Young's and shear modulus per cell
};
int static_blocks(long long ncell);
hipError_t launch_static_diag(const StaticArgs &s, double *diag, hipStream_t st);
hipError_t launch_static_start(const StaticArgs &s, const double *f, const double *diag, double *x, double *r,
                               double *z, double *p, double *partials, hipStream_t st);
hipError_t launch_static_apply(const StaticArgs &s, const double *p, double *q, double *partials, hipStream_t st);
hipError_t launch_static_step(const StaticArgs &s, double alpha, const double *p, const double *q,
                              const double *diag, double *x, double *r, double *z, double *partials,
                              hipStream_t st);
hipError_t launch_static_dir(long long ncell, double beta, const double *z, double *p, hipStream_t st);

// Largest palette whose tables fit the fused kernel's LDS.
constexpr int kFusedMaxMat = 16;
// The fused and batched kernels address all state words of one state array
// through one buffer descriptor, whose byte span must stay below 2^32.
inline bool fused_state_fits(long long stride, int tsize) {
    return (long long)N_WORDS * stride * tsize < (1LL << 32);
}

template <typename T>
hipError_t launch_fused_step(const StepArgs<T> &a, const FusedCfg &cfg, hipStream_t s);

// Batched objects: per-object descriptor and the persistent launch.
template <typename T>
struct BatchObj {
    unsigned off;           // first cell of the object in the concatenated arrays
    int nx, ny, nz;
    int tx, ty;             // tile of the object's x-y extent (tx, ty <= 64, tx * ty <= 256)
    T dt;                   // the object's stable timestep
    T origin_z;             // world z of the object's lower face
};

template <typename T>
struct BatchArgs {
    StepArgs<T> base;       // palette, parameters, material ids (concatenated)
    T *state[2];            // ping-pong state of all objects (stride = total cells)
    uint8_t *flags[2];
    const BatchObj<T> *objs;
    const int *wg_start;    // n_wg + 1 offsets into wg_objs
    const int *wg_objs;     // object ids, grouped by workgroup
    int steps;              // steps run by this launch
    int cur0;               // buffer holding the state at the first step
    long long step0;        // step index of the first step (for the time t_n)
    double temp_amp, temp_freq, temp_phase;
};

template <typename T>
hipError_t launch_batch(const BatchArgs<T> &b, int n_wg, hipStream_t s);

// Largest number of collision candidates per voxel (vx_params.contact_cap).
constexpr int kMaxContactCap = 1024;

// Collision support (self-collision on).  The voxels taking part are
// listed once (surface voxels, or all filled ones) with what the search
// needs that never changes: state index, object and packed rest indices
// within the object.  A single lattice is one object; a batch with contact
// has many, placed by their origins in one world.
struct CollideArgs {
    const int *surf_cells;       // n_surf state indices (cells), ascending within each object
    const int *surf_obj;         // n_surf object ids
    const long long *surf_ijk;   // n_surf packed rest indices within the object (21 bits per axis)
    const double *obj_origin;    // 3 per object: world position of the object's cell (0,0,0) lower corner
    int n_surf;
    int cap;                     // candidate slots per voxel
    int *cand;                   // n_surf x cap partner list indices, ascending
    int *cand_n;                 // n_surf
    unsigned *overflow;          // set when a list overflows
    unsigned *rebuild_flag;      // device flag: 1 = rebuild before next step
    unsigned *done;              // workgroups finished (last-workgroup hand-offs), 0 between launches
    double *macc;                // accumulated maximum motion
    unsigned long long *vmax_bits;
    int *cell_keys;              // n_surf hashed grid-cell keys
    long long *cell_gc;          // n_surf packed grid cells (21 bits per axis)
    // the entries of every bucket, in bucket order: list index, packed grid
    // cell, packed rest indices, object, and displacement (3 arrays of
    // n_surf values of the state precision), so that the candidate search
    // reads each entry with independent loads
    int *sorted_idx;
    long long *sorted_gc;
    long long *sorted_ijk;
    int *sorted_obj;
    void *sorted_u;
    int *bucket_start;           // table_size + 1
    int *bucket_fill;            // table_size: counts, then scatter cursors; zero between rebuilds
    int *block_sum;              // scan blocks: bucket counts per block, then their exclusive prefix;
                                 // zero between rebuilds
    int table_size;              // power of two
    unsigned long long *pair_count;  // total candidate entries
    double horizon;              // 2 l
    unsigned long long *rebuild_counter;
    Scalars *scalars;            // the block the fields above point into (motion bookkeeping)
    unsigned char *rlog;         // if set, the motion bookkeeping records there whether the step
                                 // rebuilt the lists at its start (1) or not (0)
};

// Scan blocks of a bucket table of n entries.
int scan_blocks(int n);

// Rebuild the candidate lists from the state a.s_in if the device rebuild
// flag is set; every kernel of the chain exits at once otherwise.  The
// flag stays set until the step's motion update clears it.
template <typename T>
hipError_t launch_rebuild(const StepArgs<T> &a, const CollideArgs &c, hipStream_t s);

template <typename T>
hipError_t launch_contact(const StepArgs<T> &a, const CollideArgs &c, T *contact_F, hipStream_t s);

// Motion bookkeeping after a step (one thread): closes a rebuild that ran
// at the step's start, accumulates max|v| dt, sets the rebuild flag.
template <typename T>
hipError_t launch_motion_update(const StepArgs<T> &a, const CollideArgs &c, hipStream_t s);

// Set the device rebuild flag (the next rebuild launch rebuilds).
hipError_t launch_force_rebuild(const CollideArgs &c, hipStream_t s);

// Reverse of the contact forces of one step (between the update's and the
// bonds' reverse kernels; lists valid for a.s_in).
template <typename T>
hipError_t launch_adjoint_contact(const StepArgs<T> &a, const CollideArgs &c, const AdjArgs<T> &g, hipStream_t s);

}  // namespace vx
