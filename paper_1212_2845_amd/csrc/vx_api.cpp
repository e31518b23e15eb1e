// Host side of the voxsim C ABI: validation, packing of the material grid
// into per-voxel and per-material-pair tables, timestep selection, the
// workspace carve-out and the step loop.  Device work is in the .hip files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/voxsim.h"
#include "vx_host.hpp"
#include "vx_sim.hpp"

using namespace vx;

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
template <typename T>
static void pack_tables(const vx_sim *h, std::vector<MatConst<T>> &mc, std::vector<PairConst<T>> &pc) {
    build_tables<T>(h->pal.data(), h->n_mat, h->p, mc, pc);
}

static long long cell_of(const vx_sim *h, int x, int y, int z) {
    return (long long)x + (long long)h->nx * ((long long)y + (long long)h->ny * z);
}

// Collision hash table: a power of two >= 2 x the number of cells taking
// part, and the scan scratch it needs.
static void size_collision_table(vx_sim *h) {
    int ts = 1;
    while (ts < 2 * (int)std::max<size_t>(h->coll_cells.size(), 1)) ts <<= 1;
    h->table_size = ts;
}

static void compute_layout(vx_sim *h) {
    const uint64_t n = (uint64_t)h->ncell, ts = h->tsize;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { uint64_t o = off; off = align_up(off + std::max<uint64_t>(bytes, 1)); return o; };
    Layout &L = h->L;
    L.state[0] = take(N_WORDS * n * ts);
    L.state[1] = take(N_WORDS * n * ts);
    L.mat = take(n);
    L.flags[0] = take(n);
    L.flags[1] = take(n);
    L.mats = take((uint64_t)h->n_mat * (h->precision == 64 ? sizeof(MatConst<double>) : sizeof(MatConst<float>)));
    L.pairs = take((uint64_t)h->n_mat * h->n_mat *
                   (h->precision == 64 ? sizeof(PairConst<double>) : sizeof(PairConst<float>)));
    L.bonds = take(27 * n * ts);
    L.act_amp = take(n * ts);
    L.act_phase = take(n * ts);
    L.chan = take(n);
    h->forced_cap = std::max<int>((int)h->forced_cells.size(), 1024);
    L.forced_cells = take((uint64_t)h->forced_cap * 4);
    L.forced_F = take((uint64_t)h->forced_cap * 3 * ts);
    const bool col = h->p.self_collision_on != 0;
    const uint64_t ns = col ? h->coll_cells.size() : 0;
    L.contact_F = take(col ? 3 * n * ts : 0);
    L.surf_cells = take(ns * 4);
    L.surf_obj = take(ns * 4);
    L.surf_ijk = take(ns * 8);
    L.obj_origin = take(3 * 8);
    L.cand = take(ns * (uint64_t)h->cand_cap * 4);
    L.cand_n = take(ns * 4);
    L.keys = take(ns * 4);
    L.gc = take(ns * 8);
    L.sorted = take(ns * 4);
    L.sgc = take(ns * 8);
    L.sijk = take(ns * 8);
    L.sobj = take(ns * 4);
    L.su = take(3 * ns * ts);
    L.bstart = take(col ? ((uint64_t)h->table_size + 1) * 4 : 0);
    L.bfill = take(col ? (uint64_t)h->table_size * 4 : 0);
    L.block_sum = take(col ? (uint64_t)scan_blocks(h->table_size) * 4 : 0);
    L.scalars = take(sizeof(Scalars));
    L.E_cell = take(n * ts);
    L.rho_cell = take(n * ts);
    L.energy = take((uint64_t)energy_blocks((long long)n) * kEnergyWords * 8);
    L.total = off;
}



// Upload the per-voxel, per-material and region data (not the state).
template <typename T>
static int upload_static(vx_sim *h) {
    std::vector<MatConst<T>> mc;
    std::vector<PairConst<T>> pc;
    pack_tables<T>(h, mc, pc);
    char *ws = h->ws;
    hipStream_t s = h->stream;
    HIP_OK(h, hipMemcpyAsync(ws + h->L.mat, h->grid.data(), h->ncell, hipMemcpyHostToDevice, s));
    {
        // static bits from the host, dynamic bits (friction state, contact
        // candidates) from the device copy of the current step
        std::vector<uint8_t> fl(h->flags);
        if (h->flags_live) {
            std::vector<uint8_t> dev(h->ncell);
            HIP_OK(h, hipMemcpyAsync(dev.data(), ws + h->L.flags[h->cur], h->ncell, hipMemcpyDeviceToHost, s));
            HIP_OK(h, hipStreamSynchronize(s));
            const uint8_t dyn = FLAG_STATIC | FLAG_CAND;
            for (long long c = 0; c < h->ncell; ++c) fl[c] = (uint8_t)((fl[c] & ~dyn) | (dev[c] & dyn));
        }
        HIP_OK(h, hipMemcpyAsync(ws + h->L.flags[0], fl.data(), h->ncell, hipMemcpyHostToDevice, s));
        HIP_OK(h, hipMemcpyAsync(ws + h->L.flags[1], fl.data(), h->ncell, hipMemcpyHostToDevice, s));
        HIP_OK(h, hipStreamSynchronize(s));
        h->flags_live = true;
    }
    HIP_OK(h, hipMemcpyAsync(ws + h->L.mats, mc.data(), mc.size() * sizeof(MatConst<T>), hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(ws + h->L.pairs, pc.data(), pc.size() * sizeof(PairConst<T>), hipMemcpyHostToDevice, s));
    std::vector<T> a(h->ncell), ph(h->ncell);
    if (h->has_act)
        for (long long c = 0; c < h->ncell; ++c) { a[c] = (T)h->amp[c]; ph[c] = (T)h->phase[c]; }
    HIP_OK(h, hipMemcpyAsync(ws + h->L.act_amp, a.data(), h->ncell * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(ws + h->L.act_phase, ph.data(), h->ncell * sizeof(T), hipMemcpyHostToDevice, s));
    std::vector<uint8_t> ch(h->ncell, 0);
    for (long long c = 0; c < h->ncell; ++c)
        if (h->cell_chan[c] >= 0) ch[c] = (uint8_t)h->cell_chan[c];
    HIP_OK(h, hipMemcpyAsync(ws + h->L.chan, ch.data(), h->ncell, hipMemcpyHostToDevice, s));
    // parameter mode: per-cell modulus and density, the palette's where not set
    std::vector<T> ec(h->ncell, T(0)), rc(h->ncell, T(0));
    if (h->param_mode())
        for (long long c = 0; c < h->ncell; ++c) {
            const int m = h->grid[c];
            if (!m) continue;
            ec[c] = (T)(h->has_E ? h->E_cell[c] : h->pal[m].E);
            rc[c] = (T)(h->has_rho ? h->rho_cell[c] : h->pal[m].rho);
        }
    HIP_OK(h, hipMemcpyAsync(ws + h->L.E_cell, ec.data(), h->ncell * sizeof(T), hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(ws + h->L.rho_cell, rc.data(), h->ncell * sizeof(T), hipMemcpyHostToDevice, s));
    if ((int)h->forced_cells.size() > h->forced_cap)
        return fail(h, VX_ESTATE, "more forced voxels than the workspace was sized for; set forces before the first step");
    std::vector<T> ff(h->forced_F.size());
    for (size_t i = 0; i < ff.size(); ++i) ff[i] = (T)h->forced_F[i];
    if (!h->forced_cells.empty()) {
        HIP_OK(h, hipMemcpyAsync(ws + h->L.forced_cells, h->forced_cells.data(), h->forced_cells.size() * 4, hipMemcpyHostToDevice, s));
        HIP_OK(h, hipMemcpyAsync(ws + h->L.forced_F, ff.data(), ff.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    HIP_OK(h, hipStreamSynchronize(s));
    return VX_OK;
}

template <typename T>
static int upload_state(vx_sim *h, const std::vector<double> &st) {
    std::vector<T> buf(st.size());
    for (size_t i = 0; i < st.size(); ++i) buf[i] = (T)st[i];
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[h->cur], buf.data(), buf.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    // the other buffer gets the same contents so that empty cells are defined
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[1 - h->cur], buf.data(), buf.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    return VX_OK;
}

template <typename T>
static int download_state(vx_sim *h, std::vector<double> &st) {
    std::vector<T> buf((size_t)N_WORDS * h->ncell);
    HIP_OK(h, hipMemcpyAsync(buf.data(), h->ws + h->L.state[h->cur], buf.size() * sizeof(T), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    st.resize(buf.size());
    for (size_t i = 0; i < buf.size(); ++i) st[i] = (double)buf[i];
    return VX_OK;
}

static int get_state(vx_sim *h, std::vector<double> &st) {
    if (!h->bound) { st = h->state0; return VX_OK; }
    return h->precision == 64 ? download_state<double>(h, st) : download_state<float>(h, st);
}

static int put_state(vx_sim *h, const std::vector<double> &st) {
    h->tape_valid = false;
    if (!h->bound) { h->state0 = st; return VX_OK; }
    return h->precision == 64 ? upload_state<double>(h, st) : upload_state<float>(h, st);
}

// The collision bookkeeping's rebuild threshold and every-step switch in the
// device scalars (they change with the actuation range and the scheme).
static int upload_motion_params(vx_sim *h) {
    if (!h->bound || !h->p.self_collision_on) return VX_OK;
    Scalars *sc = (Scalars *)(h->ws + h->L.scalars);
    const double thr = 2.0 * h->p.voxel_size - h->cmax;
    const unsigned every = h->coll_every ? 1u : 0u;
    HIP_OK(h, hipMemcpyAsync(&sc->threshold, &thr, sizeof(thr), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipMemcpyAsync(&sc->every, &every, sizeof(every), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    return VX_OK;
}

static int reupload_static(vx_sim *h) {
    h->tape_valid = false;
    if (!h->bound) return VX_OK;
    const int r = h->precision == 64 ? upload_static<double>(h) : upload_static<float>(h);
    return r ? r : upload_motion_params(h);
}

// Mass of filled cell c: the palette density, or the cell's own in
// parameter mode.
static double cell_mass(const vx_sim *h, long long c) {
    const double l = h->p.voxel_size;
    return (h->has_rho ? h->rho_cell[c] : h->pal[h->grid[c]].rho) * l * l * l;
}

static void update_cmax(vx_sim *h) {
    const double l = h->p.voxel_size;
    double cmax = l;
    for (long long c = 0; c < h->ncell; ++c) {
        const int m = h->grid[c];
        if (!m) continue;
        double a = std::fabs((h->flags[c] & FLAG_ACT) ? h->amp[c] : h->p.temp_amp);
        if (h->cell_chan[c] >= 0) {
            const vx_channel &ch = h->chans[h->cell_chan[c]];
            a = std::fabs(ch.offset) + std::fabs(ch.amp);
        }
        cmax = std::max(cmax, l * (1.0 + std::fabs(h->pal[m].cte) * a));
    }
    h->cmax = cmax;
}

template <typename T>
static int request_rebuild(vx_sim *h) {
    if (!h->bound || !h->p.self_collision_on) return VX_OK;
    const unsigned one = 1;
    Scalars *sc = (Scalars *)(h->ws + h->L.scalars);
    HIP_OK(h, hipMemcpyAsync(&sc->rebuild_flag, &one, sizeof(one), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    return VX_OK;
}

template <typename T>
static int enqueue_steps(vx_sim *h, int64_t n) {
    const bool col = h->p.self_collision_on != 0;
    for (int64_t i = 0; i < n; ++i) {
        StepArgs<T> a = make_args<T>(h);
        if (col) {
            CollideArgs c = make_collide(h);
            HIP_OK(h, launch_rebuild<T>(a, c, h->stream));
            HIP_OK(h, launch_contact<T>(a, c, (T *)(h->ws + h->L.contact_F), h->stream));
        }
        if (h->use_split()) {
            HIP_OK(h, launch_split_step<T>(a, h->stream));
        } else {
            HIP_OK(h, launch_fused_step<T>(a, fused_cfg(h), h->stream));
        }
        if (col) {
            CollideArgs c = make_collide(h);
            HIP_OK(h, launch_motion_update<T>(a, c, h->stream));
        }
        h->cur = 1 - h->cur;
        h->step++;
    }
    return VX_OK;
}

// Wait for the stream and report the device status flags.
static int poll_status(vx_sim *h) {
    Scalars sc;
    HIP_OK(h, hipMemcpyAsync(&sc, h->ws + h->L.scalars, sizeof(sc), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    if (sc.err_flag) return fail(h, VX_EUNSTABLE, "non-finite value in the voxel state");
    if (sc.overflow) return fail(h, VX_EOVERFLOW, "collision candidate list overflow (raise contact_cap)");
    return VX_OK;
}

template <typename T>
static int run_steps(vx_sim *h, int64_t n) {
    const int r = enqueue_steps<T>(h, n);
    return r ? r : poll_status(h);
}

template <typename T>
static int autotune(vx_sim *h, int iters, int32_t *shape_out, int32_t *zc_out) {
    const bool col = h->p.self_collision_on != 0;
    StepArgs<T> a = make_args<T>(h);
    if (col) {
        CollideArgs c = make_collide(h);
        HIP_OK(h, launch_rebuild<T>(a, c, h->stream));
        HIP_OK(h, launch_contact<T>(a, c, (T *)(h->ws + h->L.contact_F), h->stream));
    }
    hipEvent_t e0, e1;
    HIP_OK(h, hipEventCreate(&e0));
    HIP_OK(h, hipEventCreate(&e1));
    float best = 1e30f;
    FusedCfg best_cfg{0, 0, h->any_chan ? 1 : 0};
    // z chunks: the number of workgroups against the three resident per CU
    // decides the tail of the launch, so the grid is fine
    const int zcs[] = {2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 48, 64};
    for (int sh = 0; sh < kNumFusedShapes; ++sh)
        for (int zc : zcs) {
            if (zc > h->nz && zc != zcs[0]) continue;
            FusedCfg cfg{sh, zc, h->any_chan ? 1 : 0};
            // warm-up launch, then the timed ones; outputs go to the next
            // buffers and are overwritten by the first real step
            HIP_OK(h, launch_fused_step<T>(a, cfg, h->stream));
            HIP_OK(h, hipEventRecord(e0, h->stream));
            for (int i = 0; i < iters; ++i) HIP_OK(h, launch_fused_step<T>(a, cfg, h->stream));
            HIP_OK(h, hipEventRecord(e1, h->stream));
            HIP_OK(h, hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(h, hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; best_cfg = cfg; }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the timing launches touched the speed accumulator
    Scalars *sc = (Scalars *)(h->ws + h->L.scalars);
    const unsigned long long zero = 0;
    HIP_OK(h, hipMemcpyAsync(&sc->vmax_bits, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    h->fused_shape = best_cfg.shape;
    h->fused_zc = best_cfg.zc;
    if (shape_out) *shape_out = best_cfg.shape;
    if (zc_out) *zc_out = best_cfg.zc;
    return VX_OK;
}

// Average duration of the step kernel(s) alone, from the current state,
// without advancing it (same dry-run launches as the autotuner).
template <typename T>
static int time_kernel(vx_sim *h, int iters, double *ms_per_launch) {
    StepArgs<T> a = make_args<T>(h);
    if (h->p.self_collision_on) {
        CollideArgs c = make_collide(h);
        HIP_OK(h, launch_rebuild<T>(a, c, h->stream));
        HIP_OK(h, launch_contact<T>(a, c, (T *)(h->ws + h->L.contact_F), h->stream));
    }
    const bool split = h->use_split();
    const FusedCfg cfg = fused_cfg(h);
    auto launch = [&]() { return split ? launch_split_step<T>(a, h->stream) : launch_fused_step<T>(a, cfg, h->stream); };
    hipEvent_t e0, e1;
    HIP_OK(h, hipEventCreate(&e0));
    HIP_OK(h, hipEventCreate(&e1));
    HIP_OK(h, launch());
    HIP_OK(h, hipEventRecord(e0, h->stream));
    for (int i = 0; i < iters; ++i) HIP_OK(h, launch());
    HIP_OK(h, hipEventRecord(e1, h->stream));
    HIP_OK(h, hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OK(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    Scalars *sc = (Scalars *)(h->ws + h->L.scalars);
    const unsigned long long zero = 0;
    HIP_OK(h, hipMemcpyAsync(&sc->vmax_bits, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    *ms_per_launch = (double)ms / iters;
    return VX_OK;
}

template <typename T>
static int energy(vx_sim *h, double *out) {
    StepArgs<T> a = make_args<T>(h);
    double *part = (double *)(h->ws + h->L.energy);
    HIP_OK(h, launch_energy<T>(a, part, h->stream));
    const int nb = energy_blocks(h->ncell);
    std::vector<double> buf((size_t)nb * kEnergyWords);
    HIP_OK(h, hipMemcpyAsync(buf.data(), part, buf.size() * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < kEnergyWords; ++i) out[i] = 0.0;
    for (int b = 0; b < nb; ++b)
        for (int i = 0; i < kEnergyWords; ++i) out[i] += buf[(size_t)b * kEnergyWords + i];
    return VX_OK;
}

template <typename T>
static int energy_enqueue(vx_sim *h, double *out_dev) {
    StepArgs<T> a = make_args<T>(h);
    double *part = (double *)(h->ws + h->L.energy);
    HIP_OK(h, launch_energy<T>(a, part, h->stream));
    HIP_OK(h, launch_energy_sum(part, h->ncell, out_dev, h->stream));
    return VX_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int vx_create(const uint8_t *grid, int32_t nx, int32_t ny, int32_t nz, const vx_material *palette,
              int32_t n_mat, const vx_params *params, int32_t precision, void *stream, vx_handle *out) {
    VX_TRY
    if (!out) return VX_EINVAL;
    *out = nullptr;
    if (!grid || !palette || !params || nx <= 0 || ny <= 0 || nz <= 0 || n_mat < 1 || n_mat > 256)
        return VX_EINVAL;
    if (precision != 32 && precision != 64) return VX_EINVAL;
    const long long ncell = (long long)nx * ny * nz;
    if (ncell > (1LL << 31) / 16) return VX_EINVAL;
    const vx_params &p = *params;
    if (!(p.voxel_size > 0.0) || !(p.gravity >= 0.0) || !(p.zeta_bond >= 0.0) || !(p.zeta_slow >= 0.0) ||
        !(p.zeta_col >= 0.0) || !(p.dt_scale >= 0.0) || p.dt_scale > 1.0 || p.contact_cap < 0 || p.reserved != 0)
        return VX_EINVAL;
    // the collision search packs rest indices into 21 bits per axis and
    // builds each voxel's list in LDS
    if (p.self_collision_on && (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20))) return VX_EINVAL;
    if (p.contact_cap > kMaxContactCap) return VX_EINVAL;
    for (int i = 1; i < n_mat; ++i) {
        const vx_material &m = palette[i];
        if (!(m.E > 0.0) || !(m.rho > 0.0) || !(m.nu > -1.0 && m.nu < 0.5) || !(m.mu_s >= 0.0) || !(m.mu_d >= 0.0) ||
            !std::isfinite(m.cte))
            return VX_EINVAL;
    }
    for (long long c = 0; c < ncell; ++c)
        if (grid[c] >= n_mat) return VX_EINVAL;
    std::unique_ptr<vx_sim> owner(new vx_sim());
    vx_sim *h = owner.get();
    h->nx = nx; h->ny = ny; h->nz = nz; h->ncell = ncell;
    h->p = p;
    if (h->p.dt_scale == 0.0) h->p.dt_scale = 1.0;
    h->precision = precision;
    h->tsize = precision == 64 ? 8 : 4;
    h->stream = (hipStream_t)stream;
    h->n_mat = n_mat;
    h->pal.assign(palette, palette + n_mat);
    h->grid.assign(grid, grid + ncell);
    h->flags.assign(ncell, 0);
    h->amp.assign(ncell, 0.0);
    h->phase.assign(ncell, 0.0);
    h->cell_chan.assign(ncell, -1);
    h->force.assign(3 * ncell, 0.0);
    h->cand_cap = p.contact_cap > 0 ? p.contact_cap : 32;
    const double l = p.voxel_size;
    // stable timestep over bonded pairs: dt = 1 / (2 pi max sqrt(k_b / m_min))
    std::vector<char> pair_seen((size_t)n_mat * n_mat, 0);
    long long nvox = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long long c = cell_of(h, x, y, z);
                const int m = grid[c];
                if (!m) continue;
                ++nvox;
                bool surf = false;
                const int idx[3] = {x, y, z}, dim[3] = {nx, ny, nz};
                const long long stp[3] = {1, nx, (long long)nx * ny};
                for (int a = 0; a < 3; ++a) {
                    if (idx[a] == 0 || grid[c - stp[a]] == 0) surf = true;
                    if (idx[a] + 1 >= dim[a] || grid[c + stp[a]] == 0) surf = true;
                    if (idx[a] + 1 < dim[a] && grid[c + stp[a]] != 0)
                        pair_seen[(size_t)m * n_mat + grid[c + stp[a]]] = 1;
                }
                if (surf) { h->flags[c] |= FLAG_SURFACE; h->surf_cells.push_back((int)c); }
            }
    h->nvox = nvox;
    std::vector<char> seen_vox(n_mat, 0);
    for (long long c = 0; c < ncell; ++c) seen_vox[grid[c]] = 1;
    const double wmax = max_bond_omega(palette, n_mat, l, pair_seen, seen_vox);
    h->dt = wmax > 0.0 ? h->p.dt_scale / (2.0 * kPi * wmax) : 0.0;
    h->wmax = wmax;
    // rest state
    h->state0.assign((size_t)N_WORDS * ncell, 0.0);
    for (long long c = 0; c < ncell; ++c) h->state0[W_QW * ncell + c] = 1.0;
    h->coll_cells = h->surf_cells;
    size_collision_table(h);
    update_cmax(h);
    *out = owner.release();
    return VX_OK;
    VX_CATCH(nullptr)
}

int vx_workspace_bytes(vx_handle h, uint64_t *bytes) {
    VX_TRY
    if (!h || !bytes) return VX_EINVAL;
    compute_layout(h);
    *bytes = h->L.total;
    return VX_OK;
    VX_CATCH(h)
}

int vx_bind_workspace(vx_handle h, void *device_ptr, uint64_t bytes) {
    VX_TRY
    if (!h) return VX_EINVAL;
    if (h->bound) return fail(h, VX_ESTATE, "workspace already bound");
    compute_layout(h);
    if (!device_ptr || bytes < h->L.total) return fail(h, VX_EINVAL, "workspace too small");
    if (((uintptr_t)device_ptr) % kAlign) return fail(h, VX_EINVAL, "workspace not 256-byte aligned");
    h->ws = (char *)device_ptr;
    h->bound = true;
    h->cur = 0;
    int r = reupload_static(h);
    if (r != VX_OK) { h->bound = false; return r; }
    Scalars sc{};
    sc.rebuild_flag = h->p.self_collision_on ? 1u : 0u;
    sc.threshold = 2.0 * h->p.voxel_size - h->cmax;
    sc.every = h->coll_every ? 1u : 0u;
    HIP_OK(h, hipMemcpyAsync(h->ws + h->L.scalars, &sc, sizeof(sc), hipMemcpyHostToDevice, h->stream));
    if (h->p.self_collision_on) {
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_cells, h->coll_cells.data(), h->coll_cells.size() * 4,
                                 hipMemcpyHostToDevice, h->stream));
        // one object: rest indices of every listed voxel and the lattice origin
        const size_t ns = h->coll_cells.size();
        std::vector<int> obj(ns, 0);
        std::vector<long long> ijk(ns);
        for (size_t i = 0; i < ns; ++i) {
            const long long c = h->coll_cells[i];
            ijk[i] = pack_ijk((int)(c % h->nx), (int)((c / h->nx) % h->ny), (int)(c / ((long long)h->nx * h->ny)));
        }
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_obj, obj.data(), ns * 4, hipMemcpyHostToDevice, h->stream));
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_ijk, ijk.data(), ns * 8, hipMemcpyHostToDevice, h->stream));
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.obj_origin, h->p.origin, 3 * 8, hipMemcpyHostToDevice, h->stream));
        std::vector<int> zeros(ns, 0);
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.cand_n, zeros.data(), zeros.size() * 4, hipMemcpyHostToDevice, h->stream));
        std::vector<int> zt(h->table_size, 0);
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.bfill, zt.data(), zt.size() * 4, hipMemcpyHostToDevice, h->stream));
        HIP_OK(h, hipMemcpyAsync(h->ws + h->L.block_sum, zt.data(), scan_blocks(h->table_size) * 4,
                                 hipMemcpyHostToDevice, h->stream));
        HIP_OK(h, hipStreamSynchronize(h->stream));
    }
    r = put_state(h, h->state0);
    if (r != VX_OK) { h->bound = false; return r; }
    return VX_OK;
    VX_CATCH(h)
}

int vx_set_fixed(vx_handle h, const uint8_t *mask) {
    VX_TRY
    if (!h || !mask) return VX_EINVAL;
    std::vector<double> st;
    int r = get_state(h, st);
    if (r) return r;
    for (long long c = 0; c < h->ncell; ++c) {
        if (!h->grid[c]) continue;
        if (mask[c]) {
            h->flags[c] |= FLAG_FIXED;
            for (int w = W_PX; w <= W_LZ; ++w) st[(size_t)w * h->ncell + c] = 0.0;
        } else {
            h->flags[c] &= (uint8_t)~FLAG_FIXED;
        }
    }
    r = put_state(h, st);
    if (r) return r;
    return reupload_static(h);
    VX_CATCH(h)
}

static int apply_forces(vx_sim *h) {
    h->forced_cells.clear();
    h->forced_F.clear();
    for (long long c = 0; c < h->ncell; ++c) {
        h->flags[c] &= (uint8_t)~FLAG_FORCED;
        if (!h->grid[c]) continue;
        const double *f = &h->force[3 * c];
        if (f[0] != 0.0 || f[1] != 0.0 || f[2] != 0.0) {
            h->flags[c] |= FLAG_FORCED;
            h->forced_cells.push_back((int)c);
            h->forced_F.insert(h->forced_F.end(), f, f + 3);
        }
    }
    return reupload_static(h);
}

int vx_set_forces(vx_handle h, const double *force) {
    VX_TRY
    if (!h || !force) return VX_EINVAL;
    for (long long i = 0; i < 3 * h->ncell; ++i)
        if (!std::isfinite(force[i])) return fail(h, VX_EINVAL, "non-finite force");
    h->force.assign(force, force + 3 * h->ncell);
    return apply_forces(h);
    VX_CATCH(h)
}

// A voxel touches the box [lo, hi) (fractions of the workspace) when its
// cube [i/n, (i+1)/n) overlaps it with positive length on every axis.
static bool touches(const vx_sim *h, long long c, const double *loc, const double *size) {
    const int idx[3] = {(int)(c % h->nx), (int)((c / h->nx) % h->ny), (int)(c / ((long long)h->nx * h->ny))};
    const int dim[3] = {h->nx, h->ny, h->nz};
    for (int a = 0; a < 3; ++a) {
        const double lo = (double)idx[a] / dim[a], hi = (double)(idx[a] + 1) / dim[a];
        if (!(lo < loc[a] + size[a] && hi > loc[a])) return false;
    }
    return true;
}

int vx_fixed_region(vx_handle h, const double loc[3], const double size[3]) {
    VX_TRY
    if (!h || !loc || !size) return VX_EINVAL;
    std::vector<uint8_t> mask(h->ncell, 0);
    for (long long c = 0; c < h->ncell; ++c)
        mask[c] = (h->grid[c] && ((h->flags[c] & FLAG_FIXED) || touches(h, c, loc, size))) ? 1 : 0;
    return vx_set_fixed(h, mask.data());
    VX_CATCH(h)
}

int vx_forced_region(vx_handle h, const double loc[3], const double size[3], const double force[3]) {
    VX_TRY
    if (!h || !loc || !size || !force) return VX_EINVAL;
    std::vector<long long> sel;
    for (long long c = 0; c < h->ncell; ++c)
        if (h->grid[c] && touches(h, c, loc, size)) sel.push_back(c);
    if (sel.empty()) return VX_OK;
    for (long long c : sel)
        for (int k = 0; k < 3; ++k) h->force[3 * c + k] = force[k] / (double)sel.size();
    return apply_forces(h);
    VX_CATCH(h)
}

int vx_set_actuation(vx_handle h, const double *amp, const double *phase) {
    VX_TRY
    if (!h) return VX_EINVAL;
    h->has_act = amp || phase;
    for (long long c = 0; c < h->ncell; ++c) {
        h->amp[c] = amp ? amp[c] : h->p.temp_amp;
        h->phase[c] = phase ? phase[c] : h->p.temp_phase;
        if (h->has_act && h->grid[c]) h->flags[c] |= FLAG_ACT; else h->flags[c] &= (uint8_t)~FLAG_ACT;
    }
    update_cmax(h);
    return reupload_static(h);
    VX_CATCH(h)
}

int vx_set_channels(vx_handle h, const vx_channel *ch, int32_t n_ch, const int32_t *mat_channel,
                    const int32_t *cell_channel) {
    VX_TRY
    if (!h || n_ch < 0 || n_ch > VX_MAX_CHANNELS || (n_ch > 0 && !ch)) return VX_EINVAL;
    for (int k = 0; k < n_ch; ++k) {
        const vx_channel &c = ch[k];
        if (c.waveform < VX_WAVE_SINE || c.waveform > VX_WAVE_SQUARE || c.reserved != 0 ||
            !std::isfinite(c.amp) || !std::isfinite(c.freq) || !std::isfinite(c.phase) || !std::isfinite(c.offset))
            return fail(h, VX_EINVAL, "bad channel " + std::to_string(k));
    }
    std::vector<int8_t> cc(h->ncell, -1);
    for (long long c = 0; c < h->ncell; ++c) {
        if (!h->grid[c]) continue;
        int k = -1;
        if (cell_channel && cell_channel[c] >= 0) k = cell_channel[c];
        else if (mat_channel) k = mat_channel[h->grid[c]];
        if (k >= n_ch) return fail(h, VX_EINVAL, "channel index out of range at cell " + std::to_string(c));
        cc[c] = (int8_t)(k < 0 ? -1 : k);
    }
    h->chans.assign(ch, ch + n_ch);
    h->cell_chan = cc;
    h->any_chan = std::any_of(cc.begin(), cc.end(), [](int8_t k) { return k >= 0; });
    h->chan_grad_valid = false;
    for (long long c = 0; c < h->ncell; ++c) {
        if (cc[c] >= 0) h->flags[c] |= FLAG_CHAN; else h->flags[c] &= (uint8_t)~FLAG_CHAN;
    }
    h->tape_valid = false;
    update_cmax(h);
    return reupload_static(h);
    VX_CATCH(h)
}

int vx_set_velocity(vx_handle h, const double *velocity) {
    VX_TRY
    if (!h || !velocity) return VX_EINVAL;
    std::vector<double> st;
    int r = get_state(h, st);
    if (r) return r;
    for (long long c = 0; c < h->ncell; ++c) {
        if (!h->grid[c] || (h->flags[c] & FLAG_FIXED)) continue;
        const double m = cell_mass(h, c);
        for (int k = 0; k < 3; ++k) st[(size_t)(W_PX + k) * h->ncell + c] = m * velocity[3 * c + k];
    }
    return put_state(h, st);
    VX_CATCH(h)
}

int vx_step(vx_handle h, int64_t n) {
    VX_TRY
    if (!h || n < 0) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_step before vx_bind_workspace");
    if (n == 0) return VX_OK;
    h->tape_valid = false;
    return h->precision == 64 ? run_steps<double>(h, n) : run_steps<float>(h, n);
    VX_CATCH(h)
}

int vx_energy(vx_handle h, double out[10]) {
    VX_TRY
    if (!h || !out) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_energy before vx_bind_workspace");
    return h->precision == 64 ? energy<double>(h, out) : energy<float>(h, out);
    VX_CATCH(h)
}

int vx_energy_enqueue(vx_handle h, double *out) {
    VX_TRY
    if (!h || !out) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_energy_enqueue before vx_bind_workspace");
    return h->precision == 64 ? energy_enqueue<double>(h, out) : energy_enqueue<float>(h, out);
    VX_CATCH(h)
}

int vx_probe(vx_handle h, const int32_t *cells, int32_t n, int32_t word, void *out) {
    VX_TRY
    if (!h || n < 0 || word < 0 || word >= N_WORDS || (n > 0 && (!cells || !out))) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_probe before vx_bind_workspace");
    const char *st = h->ws + h->L.state[h->cur];
    if (h->precision == 64)
        HIP_OK(h, launch_probe<double>((const double *)st, h->ncell, h->ncell, cells, n, word, (double *)out,
                                       h->stream));
    else
        HIP_OK(h, launch_probe<float>((const float *)st, h->ncell, h->ncell, cells, n, word, (float *)out,
                                      h->stream));
    return VX_OK;
    VX_CATCH(h)
}

int vx_step_enqueue(vx_handle h, int64_t n) {
    VX_TRY
    if (!h || n < 0) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_step_enqueue before vx_bind_workspace");
    h->tape_valid = false;
    return h->precision == 64 ? enqueue_steps<double>(h, n) : enqueue_steps<float>(h, n);
    VX_CATCH(h)
}

int vx_status(vx_handle h) {
    VX_TRY
    if (!h) return VX_EINVAL;
    if (!h->bound) return VX_OK;
    return poll_status(h);
    VX_CATCH(h)
}

// Highest bond frequency sqrt(k_b / m_min) with per-cell moduli E and
// densities rho (NULL: the palette's); a lattice without bonds uses the
// voxels' own sqrt(E l / m).
static double param_omega(const vx_sim *h, const double *E, const double *rho) {
    const double l = h->p.voxel_size;
    const long long stp[3] = {1, h->nx, (long long)h->nx * h->ny};
    const int dim[3] = {h->nx, h->ny, h->nz};
    auto Ec = [&](long long c) { return E ? E[c] : h->pal[h->grid[c]].E; };
    auto mass = [&](long long c) { return (rho ? rho[c] : h->pal[h->grid[c]].rho) * l * l * l; };
    double w = 0.0;
    bool any_bond = false;
    for (long long c = 0; c < h->ncell; ++c) {
        if (!h->grid[c]) continue;
        const int idx[3] = {(int)(c % h->nx), (int)((c / h->nx) % h->ny), (int)(c / stp[2])};
        for (int a = 0; a < 3; ++a) {
            if (idx[a] + 1 >= dim[a] || !h->grid[c + stp[a]]) continue;
            const long long cn = c + stp[a];
            any_bond = true;
            const double kb = composite(Ec(c), Ec(cn)) * l;
            w = std::max(w, std::sqrt(kb / std::min(mass(c), mass(cn))));
        }
    }
    if (!any_bond)
        for (long long c = 0; c < h->ncell; ++c)
            if (h->grid[c]) w = std::max(w, std::sqrt(Ec(c) * l / mass(c)));
    return w;
}

// Validate and store one per-cell parameter array (dst, flag) given the
// other's current values; the timestep stays the one chosen at create, so
// no bond may become faster than the bound it was chosen for.
static int set_param(vx_sim *h, const double *vals, bool is_E, const char *what) {
    std::vector<double> &dst = is_E ? h->E_cell : h->rho_cell;
    bool &flag = is_E ? h->has_E : h->has_rho;
    if (!vals) {
        flag = false;
        dst.clear();
        return reupload_static(h);
    }
    for (long long c = 0; c < h->ncell; ++c)
        if (h->grid[c] && (!(vals[c] > 0.0) || !std::isfinite(vals[c])))
            return fail(h, VX_EINVAL, std::string("per-voxel ") + what + " must be positive and finite");
    const double *E = is_E ? vals : (h->has_E ? h->E_cell.data() : nullptr);
    const double *rho = is_E ? (h->has_rho ? h->rho_cell.data() : nullptr) : vals;
    if (param_omega(h, E, rho) > h->wmax * (1.0 + 1e-12))
        return fail(h, VX_EINVAL, std::string("per-voxel ") + what +
                                      " gives a bond above the stable bound of the timestep chosen at create");
    dst.assign(h->ncell, 0.0);
    for (long long c = 0; c < h->ncell; ++c)
        if (h->grid[c]) dst[c] = vals[c];
    flag = true;
    return reupload_static(h);
}

int vx_set_stiffness(vx_handle h, const double *E) {
    VX_TRY
    if (!h) return VX_EINVAL;
    return set_param(h, E, true, "modulus");
    VX_CATCH(h)
}

int vx_set_density(vx_handle h, const double *rho) {
    VX_TRY
    if (!h) return VX_EINVAL;
    return set_param(h, rho, false, "density");
    VX_CATCH(h)
}

int vx_read_state(vx_handle h, double *u, double *q, double *vel, double *omega) {
    VX_TRY
    if (!h) return VX_EINVAL;
    std::vector<double> st;
    int r = get_state(h, st);
    if (r) return r;
    const long long n = h->ncell;
    const double l = h->p.voxel_size;
    for (long long c = 0; c < n; ++c) {
        const int m = h->grid[c];
        const double mass = m ? cell_mass(h, c) : 1.0;
        const double I = mass * l * l / 6.0;
        for (int k = 0; k < 3; ++k) {
            if (u) u[3 * c + k] = m ? st[(size_t)(W_UX + k) * n + c] : 0.0;
            if (vel) vel[3 * c + k] = m ? st[(size_t)(W_PX + k) * n + c] / mass : 0.0;
            if (omega) omega[3 * c + k] = m ? st[(size_t)(W_LX + k) * n + c] / I : 0.0;
        }
        if (q)
            for (int k = 0; k < 4; ++k) q[4 * c + k] = m ? st[(size_t)(W_QW + k) * n + c] : (k == 0 ? 1.0 : 0.0);
    }
    return VX_OK;
    VX_CATCH(h)
}

int vx_write_state(vx_handle h, const double *u, const double *q, const double *vel, const double *omega) {
    VX_TRY
    if (!h) return VX_EINVAL;
    std::vector<double> st;
    int r = get_state(h, st);
    if (r) return r;
    const long long n = h->ncell;
    const double l = h->p.voxel_size;
    for (long long c = 0; c < n; ++c) {
        const int m = h->grid[c];
        if (!m) continue;
        const double mass = cell_mass(h, c), I = mass * l * l / 6.0;
        for (int k = 0; k < 3; ++k) {
            if (u) st[(size_t)(W_UX + k) * n + c] = u[3 * c + k];
            if (vel) st[(size_t)(W_PX + k) * n + c] = mass * vel[3 * c + k];
            if (omega) st[(size_t)(W_LX + k) * n + c] = I * omega[3 * c + k];
        }
        if (q)
            for (int k = 0; k < 4; ++k) st[(size_t)(W_QW + k) * n + c] = q[4 * c + k];
    }
    r = put_state(h, st);
    if (r) return r;
    return h->precision == 64 ? request_rebuild<double>(h) : request_rebuild<float>(h);
    VX_CATCH(h)
}

int vx_read_flags(vx_handle h, uint8_t *is_static, uint8_t *surface) {
    VX_TRY
    if (!h) return VX_EINVAL;
    std::vector<uint8_t> fl(h->flags);
    if (h->bound) {
        HIP_OK(h, hipMemcpyAsync(fl.data(), h->ws + h->L.flags[h->cur], h->ncell, hipMemcpyDeviceToHost, h->stream));
        HIP_OK(h, hipStreamSynchronize(h->stream));
    }
    for (long long c = 0; c < h->ncell; ++c) {
        if (is_static) is_static[c] = (fl[c] & FLAG_STATIC) ? 1 : 0;
        if (surface) surface[c] = (fl[c] & FLAG_SURFACE) ? 1 : 0;
    }
    return VX_OK;
    VX_CATCH(h)
}

int vx_get_dt(vx_handle h, double *dt) {
    VX_TRY
    if (!h || !dt) return VX_EINVAL;
    *dt = h->dt;
    return VX_OK;
    VX_CATCH(h)
}

int vx_get_time(vx_handle h, double *t) {
    VX_TRY
    if (!h || !t) return VX_EINVAL;
    *t = (double)h->step * h->dt;
    return VX_OK;
    VX_CATCH(h)
}

int vx_counters(vx_handle h, int64_t out[4]) {
    VX_TRY
    if (!h || !out) return VX_EINVAL;
    Scalars sc{};
    if (h->bound) {
        HIP_OK(h, hipMemcpyAsync(&sc, h->ws + h->L.scalars, sizeof(sc), hipMemcpyDeviceToHost, h->stream));
        HIP_OK(h, hipStreamSynchronize(h->stream));
    }
    out[0] = h->step;
    out[1] = (int64_t)sc.rebuilds;
    out[2] = (int64_t)sc.pair_count / 2;
    out[3] = h->nvox;
    return VX_OK;
    VX_CATCH(h)
}

int vx_candidates(vx_handle h, int32_t *cell_a, int32_t *cell_b, int32_t max_pairs, int32_t *n_pairs) {
    VX_TRY
    if (!h || !n_pairs || max_pairs < 0) return VX_EINVAL;
    *n_pairs = 0;
    if (!h->bound || !h->p.self_collision_on) return VX_OK;
    const size_t ns = h->coll_cells.size();
    std::vector<int> cand(ns * h->cand_cap), cn(ns);
    HIP_OK(h, hipMemcpyAsync(cand.data(), h->ws + h->L.cand, cand.size() * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipMemcpyAsync(cn.data(), h->ws + h->L.cand_n, cn.size() * 4, hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    int32_t k = 0;
    for (size_t i = 0; i < ns; ++i)
        for (int j = 0; j < cn[i]; ++j) {
            const int other = h->coll_cells[cand[i * h->cand_cap + j]];
            if (other <= h->coll_cells[i]) continue;
            if (k < max_pairs && cell_a && cell_b) { cell_a[k] = h->coll_cells[i]; cell_b[k] = other; }
            ++k;
        }
    *n_pairs = k;
    return VX_OK;
    VX_CATCH(h)
}

int vx_set_collision_mode(vx_handle h, int32_t all_voxels, int32_t every_step) {
    VX_TRY
    if (!h || (all_voxels != 0 && all_voxels != 1) || (every_step != 0 && every_step != 1)) return VX_EINVAL;
    if (h->bound && (all_voxels != 0) != h->coll_all)
        return fail(h, VX_ESTATE, "the voxels taking part in collision detection are fixed at bind");
    h->coll_every = every_step != 0;
    if (h->bound) {
        const int r = upload_motion_params(h);
        if (r) return r;
    }
    if (!h->bound && (all_voxels != 0) != h->coll_all) {
        h->coll_all = all_voxels != 0;
        if (h->coll_all) {
            h->coll_cells.clear();
            for (long long c = 0; c < h->ncell; ++c)
                if (h->grid[c]) h->coll_cells.push_back((int)c);
        } else {
            h->coll_cells = h->surf_cells;
        }
        size_collision_table(h);
    }
    return VX_OK;
    VX_CATCH(h)
}

int vx_set_fused_tile(vx_handle h, int32_t shape, int32_t zc) {
    VX_TRY
    if (!h || shape < -1 || shape >= kNumFusedShapes || zc < 0) return VX_EINVAL;
    h->fused_shape = shape;
    h->fused_zc = zc;
    return VX_OK;
    VX_CATCH(h)
}

int vx_get_fused_tile(vx_handle h, int32_t *shape, int32_t *tx, int32_t *ty, int32_t *zc) {
    VX_TRY
    if (!h) return VX_EINVAL;
    const FusedCfg c = fused_cfg(h);
    if (shape) *shape = c.shape;
    if (tx) *tx = kFusedShapes[c.shape].tx;
    if (ty) *ty = kFusedShapes[c.shape].ty;
    if (zc) {
        const int t = kFusedShapes[c.shape].tx, u = kFusedShapes[c.shape].ty;
        const long long cols = (long long)((h->nx + t - 1) / t) * ((h->ny + u - 1) / u);
        *zc = c.zc > 0 ? std::min(c.zc, h->nz) : balanced_zc(h->nz, cols, fused_wg_per_cu(h->precision / 8, h->param_mode()));
    }
    return VX_OK;
    VX_CATCH(h)
}

int vx_autotune(vx_handle h, int32_t iters, int32_t *shape, int32_t *zc) {
    VX_TRY
    if (!h || iters <= 0) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_autotune before vx_bind_workspace");
    if (h->n_mat > kFusedMaxMat) return fail(h, VX_ESTATE, "palette too large for the fused kernel");
    if (!fused_state_fits(h->ncell, h->precision / 8))
        return fail(h, VX_ESTATE, "lattice too large for the fused kernel");
    return h->precision == 64 ? autotune<double>(h, iters, shape, zc) : autotune<float>(h, iters, shape, zc);
    VX_CATCH(h)
}

int vx_time_kernel(vx_handle h, int32_t iters, double *ms_per_launch) {
    VX_TRY
    if (!h || iters <= 0 || !ms_per_launch) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_time_kernel before vx_bind_workspace");
    return h->precision == 64 ? time_kernel<double>(h, iters, ms_per_launch)
                              : time_kernel<float>(h, iters, ms_per_launch);
    VX_CATCH(h)
}

int vx_set_kernel(vx_handle h, int32_t kind) {
    VX_TRY
    if (!h || (kind != 0 && kind != 1)) return VX_EINVAL;
    h->kernel_kind = kind;
    return VX_OK;
    VX_CATCH(h)
}

int vx_destroy(vx_handle h) {
    VX_TRY
    delete h;
    return VX_OK;
    VX_CATCH(nullptr)
}

const char *vx_last_error(vx_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
