// Host side of differentiable rollouts (parameter mode): the forward run
// stores a checkpoint of the state every K steps; the reverse run walks the
// segments backwards, recomputes each segment's states and bond sums from
// its checkpoint with the forward kernels, then applies the reverse step
// kernels from the last step of the segment to the first.  With K = 1 the
// forward run writes every step's state, flags and bond sums straight into
// the tape (the step kernel's output goes to the next tape slot), and the
// reverse run recomputes nothing: the memory-for-time end of the trade-off,
// for rollouts whose tape fits the GPU's HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "vx_host.hpp"
#include "vx_sim.hpp"

using namespace vx;

namespace {

void grad_layout(const vx_sim *h, int64_t max_steps, int K, GradLayout &G) {
    const uint64_t n = (uint64_t)h->ncell, ts = h->tsize;
    const uint64_t sb = align_up(N_WORDS * n * ts), fb = align_up(n), fmb = align_up(6 * n * ts);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { uint64_t o = off; off = align_up(off + std::max<uint64_t>(bytes, 1)); return o; };
    G.max_steps = max_steps;
    G.K = K;
    G.n_ck = (int)((max_steps + K - 1) / K);
    G.ck_state = take(G.n_ck * sb);
    G.ck_flags = take(G.n_ck * fb);
    G.seg_state = take((uint64_t)K * sb);
    G.seg_flags = take((uint64_t)K * fb);
    G.fm = take((uint64_t)(K == 1 ? max_steps : K) * fmb);
    G.lam[0] = take(sb);
    G.lam[1] = take(sb);
    G.gfm = take(6 * n * ts);
    G.gloc = take(3 * n * ts);
    G.gE = take(n * 8);
    G.grho = take(n * 8);
    G.gphase = take(n * 8);
    G.gamp = take(n * 8);
    G.rlog = take((uint64_t)max_steps);
    G.total = off;
}

uint64_t state_slot(const vx_sim *h) { return align_up((uint64_t)N_WORDS * h->ncell * h->tsize); }
uint64_t flags_slot(const vx_sim *h) { return align_up((uint64_t)h->ncell); }
uint64_t fm_slot(const vx_sim *h) { return align_up(6ull * h->ncell * h->tsize); }

// Host staging of the reverse run: the adjoint of the state (13 words), the
// momenta words (P, L) of the first and of the final state, and the four
// FP64 per-cell gradients.
uint64_t stage_bytes(const vx_sim *h) {
    return (uint64_t)(N_WORDS + 12) * h->ncell * h->tsize + 32ull * h->ncell;
}

double voxel_mass_of(const vx_sim *h, long long c) {
    const double l = h->p.voxel_size;
    return h->has_rho ? h->rho_cell[c] * l * l * l : voxel_mass(h->pal[h->grid[c]], l);
}

template <typename T>
int grad_backward_t(vx_sim *h, const double *dL_du, const double *dL_dq, const double *dL_dv, const double *dL_dw,
                    double *g_E, double *g_rho, double *g_phase, double *g_amp, double *g_u0, double *g_q0,
                    double *g_v0, double *g_w0) {
    const GradLayout &G = h->GL;
    const long long n = h->ncell;
    const double l = h->p.voxel_size;
    char *gw = h->gws;
    hipStream_t s = h->stream;
    const uint64_t sb = state_slot(h), fb = flags_slot(h), fmb = fm_slot(h);
    // host staging (pinned when vx_grad_bind could take it)
    const size_t nz = (size_t)n, lamB = (size_t)N_WORDS * nz * sizeof(T), momB = 6 * nz * sizeof(T);
    std::unique_ptr<char[]> own_stage;
    char *stage = (char *)h->pinned;
    if (!stage || h->pinned_bytes < stage_bytes(h)) {
        own_stage.reset(new char[stage_bytes(h)]);
        stage = own_stage.get();
    }
    T *lam = (T *)stage;                                   // 13 words
    T *x0m = (T *)(stage + lamB);                          // P, L of the first state
    T *xNm = (T *)(stage + lamB + momB);                   // P, L of the final state
    double *gE = (double *)(stage + lamB + 2 * momB), *gr = gE + nz, *gp = gr + nz, *ga = gp + nz;
    // adjoint of the final state, in the stored words (v = P / m,
    // w = L / I): each group of words with a given adjoint is uploaded, the
    // others are cleared on the device
    struct Group {
        int w0, k;
        const double *src;
        int scale;   // 0: as given, 1: over m, 2: over I
    };
    const Group groups[4] = {{W_UX, 3, dL_du, 0}, {W_QW, 4, dL_dq, 0}, {W_PX, 3, dL_dv, 1}, {W_LX, 3, dL_dw, 2}};
    for (const Group &gr_ : groups) {
        T *dst = lam + (size_t)gr_.w0 * nz;
        char *dev = gw + G.lam[0] + (size_t)gr_.w0 * nz * sizeof(T);
        const size_t bytes = (size_t)gr_.k * nz * sizeof(T);
        if (!gr_.src) {
            HIP_OK(h, hipMemsetAsync(dev, 0, bytes, s));
            continue;
        }
        for (long long c = 0; c < n; ++c) {
            const bool f = h->grid[c] != 0;
            const double m = f && gr_.scale ? voxel_mass_of(h, c) : 1.0, I = m * l * l / 6.0;
            for (int k = 0; k < gr_.k; ++k) {
                const double v = gr_.src[(size_t)gr_.k * c + k];
                dst[(size_t)k * nz + c] = !f ? T(0) : gr_.scale == 1 ? (T)(v / m) : gr_.scale == 2 ? (T)(v / I) : (T)v;
            }
        }
        HIP_OK(h, hipMemcpyAsync(dev, dst, bytes, hipMemcpyHostToDevice, s));
    }
    HIP_OK(h, hipMemsetAsync(gw + G.lam[1], 0, lamB, s));
    HIP_OK(h, hipMemsetAsync(gw + G.gE, 0, n * 8, s));
    HIP_OK(h, hipMemsetAsync(gw + G.grho, 0, n * 8, s));
    HIP_OK(h, hipMemsetAsync(gw + G.gphase, 0, n * 8, s));
    HIP_OK(h, hipMemsetAsync(gw + G.gamp, 0, n * 8, s));
    int li = 0;
    const bool col = h->p.self_collision_on != 0;
    const int64_t N = h->tape_n;
    const int K = G.K;
    const int nseg = (int)((N + K - 1) / K);
    // With self-collision, candidate lists are built where the forward's
    // were: a list built at the state of step r holds every pair that
    // touches before the forward's next rebuild (the horizon rule), so one
    // list serves a piece of steps from r, or from the first step of a
    // segment (a later start within the piece, valid as long), to the next
    // rebuild; the forward logged at which steps it rebuilt.  Lists built
    // from the same state are the same, so the contact forces, and with
    // them the recomputed states, are the forward's.
    // last[k]: the forward's last rebuild at or before step k (steps
    // counted from the rollout's start), or 0
    std::vector<int64_t> last;
    if (col) {
        std::vector<unsigned char> rlog((size_t)N, 0);
        HIP_OK(h, hipMemcpyAsync(rlog.data(), gw + G.rlog, (size_t)N, hipMemcpyDeviceToHost, s));
        HIP_OK(h, hipStreamSynchronize(s));
        last.resize((size_t)N);
        for (int64_t k = 0; k < N; ++k) last[(size_t)k] = rlog[(size_t)k] ? k : (k > 0 ? last[(size_t)k - 1] : 0);
    }
    // first step of the piece of step k that begins at or after step lo
    auto piece_start = [&](int64_t k, int64_t lo) { return std::max(last[(size_t)k], lo); };
    int64_t built = -1;   // step whose state the current lists were built from
    // build the lists from state st with flags fl (into a scratch copy,
    // which receives the candidate bits and is returned)
    auto build_lists = [&](const StepArgs<T> &a, const T *st, const uint8_t *fl, uint8_t **scratch_out) -> int {
        const CollideArgs cl = make_collide(h);
        StepArgs<T> ab = a;
        ab.s_in = st;
        uint8_t *scratch = (uint8_t *)(h->ws + h->L.flags[1 - h->cur]);
        HIP_OK(h, hipMemcpyAsync(scratch, fl, (size_t)n, hipMemcpyDeviceToDevice, s));
        ab.flags = scratch;
        HIP_OK(h, launch_force_rebuild(cl, s));
        HIP_OK(h, launch_rebuild<T>(ab, cl, s));
        if (scratch_out) *scratch_out = scratch;
        return VX_OK;
    };
    for (int j = nseg - 1; j >= 0; --j) {
        const long long s0 = h->tape_step0 + (long long)j * K;
        const int len = (int)std::min<int64_t>(K, N - (int64_t)j * K);
        auto st_ptr = [&](int i) {
            return (T *)(gw + (i == 0 ? G.ck_state + (uint64_t)j * sb : G.seg_state + (uint64_t)i * sb));
        };
        auto fl_ptr = [&](int i) {
            return (uint8_t *)(gw + (i == 0 ? G.ck_flags + (uint64_t)j * fb : G.seg_flags + (uint64_t)i * fb));
        };
        // recompute the segment: states x_s0+1 .. x_s0+len-1 and the bond
        // sums of every step (the last step's new state goes to the unused
        // slot 0); with K = 1 the forward run stored them
        for (int i = 0; K > 1 && i < len; ++i) {
            StepArgs<T> a = make_args<T>(h);
            set_step_time(a, h, s0 + i);
            a.s_in = st_ptr(i);
            a.flags = fl_ptr(i);
            a.s_out = i + 1 < len ? st_ptr(i + 1) : (T *)(gw + G.seg_state);
            a.flags_out = i + 1 < len ? fl_ptr(i + 1) : (uint8_t *)(gw + G.seg_flags);
            a.fm_out = (T *)(gw + G.fm + (uint64_t)i * fmb);
            a.track_vmax = 0;
            if (col) {
                // at a piece's first step the lists are built from this
                // state, and the step reads the fresh candidate bits; later
                // steps of the piece carry them in their flags
                const int64_t k = s0 - h->tape_step0 + i;
                const int64_t start = piece_start(k, s0 - h->tape_step0);
                if (start == k) {
                    uint8_t *scratch = nullptr;
                    if (int r = build_lists(a, a.s_in, a.flags, &scratch)) return r;
                    a.flags = scratch;
                    built = k;
                }
                HIP_OK(h, launch_contact<T>(a, make_collide(h), (T *)(h->ws + h->L.contact_F), s));
            }
            if (h->use_split()) {
                HIP_OK(h, launch_split_step<T>(a, s));
            } else {
                HIP_OK(h, launch_fused_step<T>(a, fused_cfg(h), s));
            }
        }
        for (int i = len - 1; i >= 0; --i) {
            StepArgs<T> a = make_args<T>(h);
            set_step_time(a, h, s0 + i);
            a.s_in = st_ptr(i);
            a.flags = fl_ptr(i);
            a.s_out = nullptr;
            a.flags_out = nullptr;
            CollideArgs cl{};
            if (col) {
                // the lists of the step's piece (built from the piece's
                // first state, unless they already are), then the contact
                // forces at x_n; zeroed forces for voxels whose list is
                // empty, since the update's reverse reads the step's own
                // candidate bits
                cl = make_collide(h);
                const int64_t k = s0 - h->tape_step0 + i;
                const int64_t lo = K > 1 ? s0 - h->tape_step0 : 0;
                const int64_t start = piece_start(k, lo);
                if (start != built) {
                    const T *st = K > 1 ? st_ptr((int)(start - lo))
                                        : (const T *)(gw + G.ck_state + (uint64_t)start * sb);
                    const uint8_t *fl = K > 1 ? fl_ptr((int)(start - lo))
                                              : (const uint8_t *)(gw + G.ck_flags + (uint64_t)start * fb);
                    if (int r = build_lists(a, st, fl, nullptr)) return r;
                    built = start;
                }
                HIP_OK(h, hipMemsetAsync(h->ws + h->L.contact_F, 0, (size_t)3 * n * sizeof(T), s));
                HIP_OK(h, launch_contact<T>(a, cl, (T *)(h->ws + h->L.contact_F), s));
            }
            AdjArgs<T> g;
            g.fm = (const T *)(gw + G.fm + (uint64_t)(K > 1 ? i : j) * fmb);
            g.lam_in = (const T *)(gw + G.lam[li]);
            g.lam_out = (T *)(gw + G.lam[1 - li]);
            g.gfm = (T *)(gw + G.gfm);
            g.gloc = (T *)(gw + G.gloc);
            g.g_E = (double *)(gw + G.gE);
            g.g_rho = (double *)(gw + G.grho);
            g.g_phase = (double *)(gw + G.gphase);
            g.g_amp = (double *)(gw + G.gamp);
            set_chan_derivs(g.chan_dph, g.chan_dam, h, s0 + i);
            HIP_OK(h, launch_adjoint_step<T>(a, g, col ? &cl : nullptr, s));
            li = 1 - li;
        }
    }
    if (col) {
        // the lists now hold the first step's pairs: rebuild before the next
        HIP_OK(h, launch_force_rebuild(make_collide(h), s));
    }
    HIP_OK(h, hipMemcpyAsync(lam, gw + G.lam[li], lamB, hipMemcpyDeviceToHost, s));
    // momenta of the initial state (checkpoint 0) and of the final state,
    // for the density's effect through the conversions between momenta and
    // velocities: the initial velocities are held fixed (P0 = m v0) and the
    // loss reads the final velocities (v = P / m); P and L are words 7-12
    const bool want_xN = g_rho && (dL_dv || dL_dw);
    const size_t mom0 = (size_t)W_PX * nz * sizeof(T);
    if (g_rho) HIP_OK(h, hipMemcpyAsync(x0m, gw + G.ck_state + mom0, momB, hipMemcpyDeviceToHost, s));
    if (want_xN) HIP_OK(h, hipMemcpyAsync(xNm, h->ws + h->L.state[h->cur] + mom0, momB, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipMemcpyAsync(gE, gw + G.gE, nz * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipMemcpyAsync(gr, gw + G.grho, nz * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipMemcpyAsync(gp, gw + G.gphase, nz * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipMemcpyAsync(ga, gw + G.gamp, nz * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    Scalars sc;
    HIP_OK(h, hipMemcpyAsync(&sc, h->ws + h->L.scalars, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    if (sc.err_flag) return fail(h, VX_EUNSTABLE, "non-finite value in the voxel state");
    if (sc.overflow) return fail(h, VX_EOVERFLOW, "collision candidate list overflow (raise contact_cap)");
    // channel voxels: their terms summed per channel in cell order, and
    // zero in the per-voxel outputs
    h->chan_gphase.assign(h->chans.size(), 0.0);
    h->chan_gamp.assign(h->chans.size(), 0.0);
    for (long long c = 0; c < n; ++c) {
        if (!h->grid[c] || h->cell_chan[c] < 0) continue;
        h->chan_gphase[h->cell_chan[c]] += gp[c];
        h->chan_gamp[h->cell_chan[c]] += ga[c];
        gp[c] = ga[c] = 0.0;
    }
    h->chan_grad_valid = true;
    const bool need_m = g_rho || g_v0 || g_w0;
    for (long long c = 0; c < n; ++c) {
        const bool f = h->grid[c] != 0;
        const double m = f && need_m ? voxel_mass_of(h, c) : 0.0, I = m * l * l / 6.0;
        if (g_E) g_E[c] = f ? gE[c] : 0.0;
        if (g_rho) {
            // P0 = m v0 and L0 = I w0 with m, I proportional to rho
            double gi = 0.0;
            if (f) {
                const double rho = m / (l * l * l);
                for (int k = 0; k < 3; ++k) {
                    gi += (double)lam[(size_t)(W_PX + k) * n + c] * (double)x0m[(size_t)k * n + c] +
                          (double)lam[(size_t)(W_LX + k) * n + c] * (double)x0m[(size_t)(3 + k) * n + c];
                    if (dL_dv) gi -= dL_dv[3 * c + k] * (double)xNm[(size_t)k * n + c] / m;
                    if (dL_dw) gi -= dL_dw[3 * c + k] * (double)xNm[(size_t)(3 + k) * n + c] / I;
                }
                gi /= rho;
            }
            g_rho[c] = f ? gr[c] + gi : 0.0;
        }
        if (g_phase) g_phase[c] = f ? gp[c] : 0.0;
        if (g_amp) g_amp[c] = f ? ga[c] : 0.0;
        for (int k = 0; k < 3; ++k) {
            if (g_u0) g_u0[3 * c + k] = f ? (double)lam[(size_t)(W_UX + k) * n + c] : 0.0;
            if (g_v0) g_v0[3 * c + k] = f ? (double)lam[(size_t)(W_PX + k) * n + c] * m : 0.0;
            if (g_w0) g_w0[3 * c + k] = f ? (double)lam[(size_t)(W_LX + k) * n + c] * I : 0.0;
        }
        if (g_q0)
            for (int k = 0; k < 4; ++k) g_q0[4 * c + k] = f ? (double)lam[(size_t)(W_QW + k) * n + c] : 0.0;
    }
    return VX_OK;
}

template <typename T>
int checkpoint(vx_sim *h, int j);

// Forward run with K = 1: step j reads tape slot j and writes slot j + 1
// (the last step writes the handle's next state buffer) and its bond sums
// to bond-sum slot j.
template <typename T>
int tape_forward(vx_sim *h, int64_t n) {
    const GradLayout &G = h->GL;
    const uint64_t sb = state_slot(h), fb = flags_slot(h), fmb = fm_slot(h);
    char *gw = h->gws;
    int r = checkpoint<T>(h, 0);
    if (r) return r;
    for (int64_t j = 0; j < n; ++j) {
        StepArgs<T> a = make_args<T>(h);
        const bool last = j + 1 == n;
        a.s_in = (const T *)(gw + G.ck_state + (uint64_t)j * sb);
        a.flags = (const uint8_t *)(gw + G.ck_flags + (uint64_t)j * fb);
        a.s_out = last ? (T *)(h->ws + h->L.state[1 - h->cur]) : (T *)(gw + G.ck_state + (uint64_t)(j + 1) * sb);
        a.flags_out = last ? (uint8_t *)(h->ws + h->L.flags[1 - h->cur])
                           : (uint8_t *)(gw + G.ck_flags + (uint64_t)(j + 1) * fb);
        a.fm_out = (T *)(gw + G.fm + (uint64_t)j * fmb);
        const bool col = h->p.self_collision_on != 0;
        CollideArgs cl{};
        if (col) {
            cl = make_collide(h);
            HIP_OK(h, launch_rebuild<T>(a, cl, h->stream));
            HIP_OK(h, launch_contact<T>(a, cl, (T *)(h->ws + h->L.contact_F), h->stream));
        }
        if (h->use_split()) {
            HIP_OK(h, launch_split_step<T>(a, h->stream));
        } else {
            HIP_OK(h, launch_fused_step<T>(a, fused_cfg(h), h->stream));
        }
        if (col) HIP_OK(h, launch_motion_update<T>(a, cl, h->stream));
        h->step++;
    }
    h->cur = 1 - h->cur;
    Scalars sc;
    HIP_OK(h, hipMemcpyAsync(&sc, h->ws + h->L.scalars, sizeof(sc), hipMemcpyDeviceToHost, h->stream));
    HIP_OK(h, hipStreamSynchronize(h->stream));
    if (sc.err_flag) return fail(h, VX_EUNSTABLE, "non-finite value in the voxel state");
    if (sc.overflow) return fail(h, VX_EOVERFLOW, "collision candidate list overflow (raise contact_cap)");
    return VX_OK;
}

template <typename T>
int checkpoint(vx_sim *h, int j) {
    const uint64_t sb = state_slot(h), fb = flags_slot(h);
    HIP_OK(h, hipMemcpyAsync(h->gws + h->GL.ck_state + (uint64_t)j * sb, h->ws + h->L.state[h->cur],
                             (size_t)N_WORDS * h->ncell * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
    HIP_OK(h, hipMemcpyAsync(h->gws + h->GL.ck_flags + (uint64_t)j * fb, h->ws + h->L.flags[h->cur], h->ncell,
                             hipMemcpyDeviceToDevice, h->stream));
    return VX_OK;
}

}  // namespace

extern "C" {

int vx_grad_workspace_bytes(vx_handle h, int64_t max_steps, int32_t K, uint64_t *bytes) {
    VX_TRY
    if (!h || !bytes || max_steps < 1 || K < 1) return VX_EINVAL;
    GradLayout G;
    grad_layout(h, max_steps, std::min<int64_t>(K, max_steps), G);
    *bytes = G.total;
    return VX_OK;
    VX_CATCH(h)
}

int vx_grad_bind(vx_handle h, void *device_ptr, uint64_t bytes, int64_t max_steps, int32_t K) {
    VX_TRY
    if (!h || max_steps < 1 || K < 1) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_grad_bind before vx_bind_workspace");
    GradLayout G;
    grad_layout(h, max_steps, (int)std::min<int64_t>(K, max_steps), G);
    if (!device_ptr || bytes < G.total) return fail(h, VX_EINVAL, "gradient workspace too small");
    if (((uintptr_t)device_ptr) % kAlign) return fail(h, VX_EINVAL, "gradient workspace not 256-byte aligned");
    h->gws = (char *)device_ptr;
    h->GL = G;
    h->tape_valid = false;
    if (h->pinned_bytes < stage_bytes(h)) {
        if (h->pinned) (void)hipHostFree(h->pinned);
        h->pinned = nullptr;
        h->pinned_bytes = 0;
        void *p = nullptr;
        if (hipHostMalloc(&p, stage_bytes(h), hipHostMallocDefault) == hipSuccess) {
            h->pinned = p;
            h->pinned_bytes = stage_bytes(h);
        } else {
            (void)hipGetLastError();   // the reverse run stages in ordinary host memory
        }
    }
    return VX_OK;
    VX_CATCH(h)
}

int vx_set_stiffness(vx_handle h, const double *E);

int vx_grad_forward(vx_handle h, int64_t n) {
    VX_TRY
    if (!h || n < 1) return VX_EINVAL;
    if (!h->gws) return fail(h, VX_ESTATE, "vx_grad_forward before vx_grad_bind");
    if (n > h->GL.max_steps) return fail(h, VX_EINVAL, "more steps than the gradient workspace was sized for");
    if (!h->param_mode()) {
        // parameter mode with the palette's moduli (and densities)
        std::vector<double> E(h->ncell, 0.0);
        for (long long c = 0; c < h->ncell; ++c)
            if (h->grid[c]) E[c] = h->pal[h->grid[c]].E;
        const int r = vx_set_stiffness(h, E.data());
        if (r) return r;
    }
    const long long step0 = h->step;
    const int K = h->GL.K;
    // the motion bookkeeping of every step logs whether the step rebuilt
    // the candidate lists, which the reverse run follows
    struct LogOn {   // the log is on for this call only, whatever ends it
        vx_sim *h;
        ~LogOn() { h->rlog = nullptr; }
    } log_on{h};
    h->rlog = (unsigned char *)(h->gws + h->GL.rlog);
    h->rlog_step0 = step0;
    h->rlog_n = n;
    int r = 0;
    if (K == 1) r = h->precision == 64 ? tape_forward<double>(h, n) : tape_forward<float>(h, n);
    for (int64_t done = 0, j = 0; !r && K > 1 && done < n; done += K, ++j) {
        r = h->precision == 64 ? checkpoint<double>(h, (int)j) : checkpoint<float>(h, (int)j);
        if (!r) r = vx_step(h, std::min<int64_t>(K, n - done));
    }
    if (r) return r;
    h->tape_valid = true;
    h->tape_n = n;
    h->tape_step0 = step0;
    return VX_OK;
    VX_CATCH(h)
}

int vx_grad_backward(vx_handle h, const double *dL_du, const double *dL_dq, const double *dL_dv, const double *dL_dw,
                     double *g_E, double *g_rho, double *g_phase, double *g_amp, double *g_u0, double *g_q0,
                     double *g_v0, double *g_w0) {
    VX_TRY
    if (!h) return VX_EINVAL;
    if (!h->tape_valid || h->step != h->tape_step0 + h->tape_n)
        return fail(h, VX_ESTATE, "no recorded rollout ends at the current state (vx_grad_forward first)");
    return h->precision == 64
               ? grad_backward_t<double>(h, dL_du, dL_dq, dL_dv, dL_dw, g_E, g_rho, g_phase, g_amp, g_u0, g_q0, g_v0,
                                         g_w0)
               : grad_backward_t<float>(h, dL_du, dL_dq, dL_dv, dL_dw, g_E, g_rho, g_phase, g_amp, g_u0, g_q0, g_v0,
                                        g_w0);
    VX_CATCH(h)
}

int vx_grad_channels(vx_handle h, double *g_phase, double *g_amp) {
    VX_TRY
    if (!h) return VX_EINVAL;
    if (!h->chan_grad_valid || h->chan_gphase.size() != h->chans.size())
        return fail(h, VX_ESTATE, "vx_grad_channels before vx_grad_backward with the current channels");
    for (size_t k = 0; k < h->chans.size(); ++k) {
        if (g_phase) g_phase[k] = h->chan_gphase[k];
        if (g_amp) g_amp[k] = h->chan_gamp[k];
    }
    return VX_OK;
    VX_CATCH(h)
}

}  // extern "C"
