// Internal state of one single-lattice handle and the helpers shared by the
// host files that implement its C ABI (plain stepping and differentiable
// rollouts).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/voxsim.h"
#include "vx_launch.hpp"
#include "vx_types.hpp"

namespace vx {

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    uint64_t state[2], mat, flags[2], mats, pairs, bonds, act_amp, act_phase, chan, forced_cells, forced_F;
    uint64_t contact_F, surf_cells, surf_obj, surf_ijk, obj_origin, cand, cand_n, keys, gc, sorted, sgc, sijk,
        sobj, su, bstart, bfill, block_sum, scalars;
    uint64_t E_cell, rho_cell;
    uint64_t energy;
    uint64_t total;
};

// Carve-out of the caller's gradient workspace for a rollout of up to
// max_steps steps with a checkpoint every K steps.
struct GradLayout {
    int64_t max_steps;
    int K;
    int n_ck;                    // checkpoints: states at steps 0, K, 2K, ...
    uint64_t ck_state, ck_flags; // n_ck x (13 words x ncell), n_ck x ncell bytes
    uint64_t seg_state, seg_flags; // K slots: states of one segment (slot 0 unused)
    uint64_t fm;                 // K slots x 6 words x ncell: bond sums of each segment step
    uint64_t lam[2];             // adjoint state, 13 words x ncell each
    uint64_t gfm;                // adjoint of the bond sums, 6 words x ncell
    uint64_t gloc;               // per-voxel adjoints of strain, modulus and mass from the update, 3 x ncell
    uint64_t gE, grho, gphase, gamp;   // FP64 accumulators, ncell each
    uint64_t rlog;               // max_steps bytes: 1 where the forward rebuilt the candidate lists
    uint64_t total;
};



}  // namespace vx

using namespace vx;

struct vx_sim {
    int nx = 0, ny = 0, nz = 0;
    long long ncell = 0;
    vx_params p{};
    int precision = 64;
    size_t tsize = 8;
    hipStream_t stream = nullptr;
    int n_mat = 0;
    std::vector<vx_material> pal;
    std::vector<uint8_t> grid, flags;
    std::vector<double> amp, phase;      // per cell; valid where FLAG_ACT
    bool has_act = false;
    // named actuation channels and each cell's channel (-1: none)
    std::vector<vx_channel> chans;
    std::vector<int8_t> cell_chan;
    bool any_chan = false;            // some filled cell follows a channel
    // per-channel gradients of the last reverse run
    std::vector<double> chan_gphase, chan_gamp;
    bool chan_grad_valid = false;
    std::vector<double> force;           // ncell x 3 (host copy)
    std::vector<int> forced_cells;
    std::vector<double> forced_F;
    int forced_cap = 0;
    std::vector<int> surf_cells;
    // collision detection: the cells that take part (the surface voxels, or
    // every filled voxel), and whether candidates are rebuilt every step
    // instead of when the accumulated motion reaches the horizon rule
    std::vector<int> coll_cells;
    bool coll_all = false, coll_every = false;
    long long nvox = 0;
    double dt = 0.0;
    long long step = 0;
    int kernel_kind = 0;
    int cand_cap = 32;
    int table_size = 1;
    double cmax = 0.0;
    // initial state in double, 13 x ncell (used until bind)
    std::vector<double> state0;
    // device
    bool bound = false;
    char *ws = nullptr;
    Layout L{};
    int cur = 0;                          // which state / flags buffer holds step n
    bool flags_live = false;              // device flags hold dynamic bits
    int fused_shape = -1;                 // tile shape of the fused kernel (-1: heuristic)
    int fused_zc = 0;                     // z chunk of the fused kernel (0: heuristic)
    // parameter mode: per-cell elastic modulus and density; a quantity not
    // set per cell takes its palette value
    bool has_E = false, has_rho = false;
    std::vector<double> E_cell, rho_cell;
    bool param_mode() const { return has_E || has_rho; }
    // the split kernels run when asked for, for palettes over 16 materials
    // and for state arrays beyond the fused kernel's span
    bool use_split() const {
        return kernel_kind == 1 || n_mat > vx::kFusedMaxMat || !vx::fused_state_fits(ncell, precision / 8);
    }
    double wmax = 0.0;                    // sqrt(k_b / m_min) the timestep was chosen for
    // differentiable rollouts
    char *gws = nullptr;
    vx::GradLayout GL{};
    bool tape_valid = false;              // a recorded rollout ends at the current state
    int64_t tape_n = 0;
    long long tape_step0 = 0;
    // while a recorded forward runs: its rebuild log (device), first step
    // and length
    unsigned char *rlog = nullptr;
    long long rlog_step0 = 0;
    int64_t rlog_n = 0;
    // pinned host memory for the reverse run's host copies (taken at
    // vx_grad_bind when it can be; ordinary host memory otherwise)
    void *pinned = nullptr;
    uint64_t pinned_bytes = 0;
    std::string err;

    vx_sim() = default;
    vx_sim(const vx_sim &) = delete;
    vx_sim &operator=(const vx_sim &) = delete;
    ~vx_sim() {
        if (pinned) (void)hipHostFree(pinned);
    }
};

inline int fail(vx_sim *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

#define HIP_OK(h, call)                                                        \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            return fail(h, VX_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// A channel's waveform at phase angle theta and its derivative with
// respect to theta.  Triangle and square are in phase with the sine: the
// triangle rises from 0 to its peak over the first quarter period, the
// square is +1 over the first half period.
inline void channel_wave(int waveform, double theta, double *w, double *dw) {
    if (waveform == VX_WAVE_SINE) {
        *w = std::sin(theta);
        *dw = std::cos(theta);
        return;
    }
    const double turns = theta / (2.0 * vx::kPi);
    const double x = turns - std::floor(turns);   // position in the period, [0, 1)
    if (waveform == VX_WAVE_TRIANGLE) {
        const double slope = 4.0 / (2.0 * vx::kPi);   // 4 per period, per radian
        if (x < 0.25) { *w = 4.0 * x; *dw = slope; }
        else if (x < 0.75) { *w = 2.0 - 4.0 * x; *dw = -slope; }
        else { *w = 4.0 * x - 4.0; *dw = slope; }
        return;
    }
    *w = x < 0.5 ? 1.0 : -1.0;
    *dw = 0.0;
}

// Time-dependent fields of the step arguments at step index n (t_n = n dt).
template <typename T>
inline void set_step_time(vx::StepArgs<T> &a, const vx_sim *h, long long n) {
    const double tn = (double)n * h->dt;
    const double wt = 2.0 * vx::kPi * h->p.temp_freq * tn;
    a.wt = wt;
    a.wt_red = (T)std::fmod(wt, 2.0 * vx::kPi);
    a.dT_global = (T)(h->p.temp_amp * std::sin(wt + h->p.temp_phase));
    a.chan_dT = vx::Chan8<T>{};
    for (int k = 0; k < (int)h->chans.size() && k < vx::kMaxChan; ++k) {
        const vx_channel &c = h->chans[k];
        double w, dw;
        channel_wave(c.waveform, 2.0 * vx::kPi * c.freq * tn + c.phase, &w, &dw);
        vx::chan_set(a.chan_dT, k, (T)(c.offset + c.amp * w));
    }
}

// The channels' temperature derivatives at step index n, for the reverse
// step: with respect to each channel's phase and amplitude.
template <typename T>
inline void set_chan_derivs(vx::Chan8<T> &dph, vx::Chan8<T> &dam, const vx_sim *h, long long n) {
    const double tn = (double)n * h->dt;
    dph = dam = vx::Chan8<T>{};
    for (int k = 0; k < (int)h->chans.size() && k < vx::kMaxChan; ++k) {
        const vx_channel &c = h->chans[k];
        double w, dw;
        channel_wave(c.waveform, 2.0 * vx::kPi * c.freq * tn + c.phase, &w, &dw);
        vx::chan_set(dph, k, (T)(c.amp * dw));
        vx::chan_set(dam, k, (T)w);
    }
}

template <typename T>
inline vx::StepArgs<T> make_args(vx_sim *h) {
    StepArgs<T> a{};
    char *ws = h->ws;
    a.s_in = (const T *)(ws + h->L.state[h->cur]);
    a.s_out = (T *)(ws + h->L.state[1 - h->cur]);
    a.stride = h->ncell;
    a.mat = (const uint8_t *)(ws + h->L.mat);
    a.flags = (const uint8_t *)(ws + h->L.flags[h->cur]);
    a.flags_out = (uint8_t *)(ws + h->L.flags[1 - h->cur]);
    a.mats = (const MatConst<T> *)(ws + h->L.mats);
    a.pairs = (const PairConst<T> *)(ws + h->L.pairs);
    a.n_mat = h->n_mat;
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz;
    a.l = (T)h->p.voxel_size;
    a.dt = (T)h->dt;
    a.gravity = (T)h->p.gravity;
    a.origin_z = (T)h->p.origin[2];
    for (int k = 0; k < 3; ++k) a.origin[k] = h->p.origin[k];
    set_step_time(a, h, h->step);
    a.act_amp = (const T *)(ws + h->L.act_amp);
    a.act_phase = (const T *)(ws + h->L.act_phase);
    a.chan = (const uint8_t *)(ws + h->L.chan);
    a.forced_cells = (const int *)(ws + h->L.forced_cells);
    a.forced_F = (const T *)(ws + h->L.forced_F);
    a.n_forced = (int)h->forced_cells.size();
    a.floor_on = h->p.floor_on;
    a.track_vmax = h->p.self_collision_on;
    a.contact_F = (const T *)(ws + h->L.contact_F);
    a.bonds = (T *)(ws + h->L.bonds);
    a.E_cell = h->param_mode() ? (const T *)(ws + h->L.E_cell) : nullptr;
    a.rho_cell = h->param_mode() ? (const T *)(ws + h->L.rho_cell) : nullptr;
    a.fm_out = nullptr;
    a.zeta_bond = (T)h->p.zeta_bond;
    a.zeta_slow = (T)h->p.zeta_slow;
    a.zeta_col = (T)h->p.zeta_col;
    Scalars *sc = (Scalars *)(ws + h->L.scalars);
    a.err_flag = &sc->err_flag;
    a.vmax_bits = &sc->vmax_bits;
    return a;
}

inline vx::CollideArgs make_collide(vx_sim *h) {
    CollideArgs c{};
    char *ws = h->ws;
    c.surf_cells = (const int *)(ws + h->L.surf_cells);
    c.surf_obj = (const int *)(ws + h->L.surf_obj);
    c.surf_ijk = (const long long *)(ws + h->L.surf_ijk);
    c.obj_origin = (const double *)(ws + h->L.obj_origin);
    c.n_surf = (int)h->coll_cells.size();
    c.cap = h->cand_cap;
    c.cand = (int *)(ws + h->L.cand);
    c.cand_n = (int *)(ws + h->L.cand_n);
    Scalars *sc = (Scalars *)(ws + h->L.scalars);
    c.overflow = &sc->overflow;
    c.rebuild_flag = &sc->rebuild_flag;
    c.done = &sc->done;
    c.macc = &sc->macc;
    c.vmax_bits = &sc->vmax_bits;
    c.cell_keys = (int *)(ws + h->L.keys);
    c.cell_gc = (long long *)(ws + h->L.gc);
    c.sorted_idx = (int *)(ws + h->L.sorted);
    c.sorted_gc = (long long *)(ws + h->L.sgc);
    c.sorted_ijk = (long long *)(ws + h->L.sijk);
    c.sorted_obj = (int *)(ws + h->L.sobj);
    c.sorted_u = (void *)(ws + h->L.su);
    c.bucket_start = (int *)(ws + h->L.bstart);
    c.bucket_fill = (int *)(ws + h->L.bfill);
    c.block_sum = (int *)(ws + h->L.block_sum);
    c.table_size = h->table_size;
    c.pair_count = &sc->pair_count;
    c.horizon = 2.0 * h->p.voxel_size;
    c.rebuild_counter = &sc->rebuilds;
    c.scalars = sc;
    const long long k = h->step - h->rlog_step0;
    c.rlog = h->rlog && k >= 0 && k < h->rlog_n ? h->rlog + k : nullptr;
    return c;
}

// Tile shape of the fused kernel: the one wasting the fewest lanes on the
// lattice's x-y extent, with the ring (halo) and boundary-bond overhead of
// small tiles as a tie breaker.
inline int heuristic_shape(const vx_sim *h) {
    int best = 0;
    double best_cost = 1e300;
    for (int i = 0; i < vx::kNumFusedShapes; ++i) {
        const int tx = vx::kFusedShapes[i].tx, ty = vx::kFusedShapes[i].ty;
        const double padded = (double)((h->nx + tx - 1) / tx * tx) * (double)((h->ny + ty - 1) / ty * ty);
        const double slots = padded / ((double)h->nx * h->ny);
        const double halo = 2.0 * (tx + ty) / (double)(tx * ty);
        const double cost = slots * (1.0 + 0.3 * halo);
        if (cost < best_cost - 1e-12) { best_cost = cost; best = i; }
    }
    return best;
}

// Launch configuration of the fused step kernel: the chosen or heuristic
// tile shape, the z chunk, and whether any voxel follows a named channel.
inline vx::FusedCfg fused_cfg(const vx_sim *h) {
    vx::FusedCfg c;
    c.shape = h->fused_shape >= 0 ? h->fused_shape : heuristic_shape(h);
    c.zc = h->fused_zc;
    c.chan = h->any_chan ? 1 : 0;
    return c;
}
