// Host side of the batched C ABI: many voxel objects packed into one set of
// arrays.  Independent objects are stepped by one persistent launch, each
// with its own stable timestep (Eq. 31-32 over its own bonds); with contact
// on, the objects share one world, one timestep and one surface hash, and
// every step runs the collision chain, the contact forces and one launch of
// the batch kernel.  Each object's x-y footprint is cut into tiles by one of
// two rules, objects are assigned to workgroups by longest-processing-time
// packing on cell count, and the autotuner times both rules over a range of
// workgroup counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "../../include/voxsim.h"
#include "vx_host.hpp"
#include "vx_launch.hpp"
#include "vx_types.hpp"

using namespace vx;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct ObjHost {
    long long off;
    int nx, ny, nz;
    int tx, ty;                  // the tile in force
    int tile[2][2];              // the tile of each rule
    double dt;
    double origin_z;
    long long nvox;
};

// Tiles of the batch kernel: TX, TY <= 64 and TX TY <= 256 (one 256-lane
// workgroup, lane t at x = t mod TX, y = t / TX of the tile, marching the
// object's height).  Rows as wide as the footprint keep each wavefront's
// loads on few, long runs of cells, and fewer tiles mean fewer ring cells
// loaded; narrower tiles that leave fewer lanes idle lost on both counts.
// Rule 0: TX = min(nx, 64), then as many rows as fit.
// Rule 1: as many tiles across x as rule 0, evened out (a footprint 70
// wide takes two tiles of 35, not 64 and 6), then as many rows as fit.
constexpr int kTileRules = 2;

void choose_tiles(ObjHost &o) {
    o.tile[0][0] = std::min(o.nx, 64);
    o.tile[0][1] = std::min(std::min(o.ny, 256 / o.tile[0][0]), 64);
    const int across = (o.nx + 63) / 64;
    o.tile[1][0] = (o.nx + across - 1) / across;
    o.tile[1][1] = std::min(std::min(o.ny, 256 / o.tile[1][0]), 64);
}

}  // namespace

struct vx_batch_sim {
    int precision = 32;
    size_t tsize = 4;
    hipStream_t stream = nullptr;
    vx_params p{};
    int n_mat = 0;
    std::vector<vx_material> pal;
    std::vector<ObjHost> objs;
    std::vector<uint8_t> grid;   // concatenated material ids
    long long total = 0;         // cells
    long long nvox = 0;
    int n_wg = 0;                // workgroups of the persistent launch (0: default)
    int tile_rule = 0;           // how the objects' footprints are tiled
    int max_steps_per_launch = 2000;
    long long step = 0;
    int cur = 0;
    bool bound = false;
    char *ws = nullptr;
    struct {
        uint64_t state[2], mat, flags[2], mats, pairs, objs, wg_start, wg_objs, scalars, total;
        // contact between objects
        uint64_t contact_F, surf_cells, surf_obj, surf_ijk, obj_origin, cand, cand_n, keys, gc, sorted, sgc, sijk,
            sobj, su, bstart, bfill, block_sum;
    } L{};
    int wg_cap = 0;              // capacity of the workgroup tables
    // contact: the surface voxels of every object (state index, object,
    // rest indices), the objects' origins, the candidate capacity, the hash
    // table size and the largest contact size actuation can produce
    bool contact = false;
    std::vector<int> surf_cells, surf_obj;
    std::vector<long long> surf_ijk;
    std::vector<double> origins;
    int cand_cap = 32;
    int table_size = 1;
    double cmax = 0.0;
    double dt = 0.0;             // the common timestep with contact
    std::string err;
};

static int bfail(vx_batch_sim *h, int code, const std::string &m) {
    if (h) h->err = m;
    return code;
}

#define BHIP_OK(h, call)                                                                 \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return bfail(h, VX_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static void pack_tables(const vx_batch_sim *h, std::vector<MatConst<T>> &mc, std::vector<PairConst<T>> &pc) {
    build_tables<T>(h->pal.data(), h->n_mat, h->p, mc, pc);
}

static int default_wg(const vx_batch_sim *h) {
    // one workgroup per object: the hardware hands each free slot the next
    // object in packing order (largest first), which balanced the
    // 4096-object mix better than any static packing of fewer workgroups
    return (int)std::min<size_t>(h->objs.size(), (size_t)INT32_MAX);
}

static void layout(vx_batch_sim *h) {
    const uint64_t n = (uint64_t)h->total, ts = h->tsize;
    uint64_t off = 0;
    auto take = [&](uint64_t b) { uint64_t o = off; off = align_up(off + std::max<uint64_t>(b, 1)); return o; };
    h->L.state[0] = take(N_WORDS * n * ts);
    h->L.state[1] = take(N_WORDS * n * ts);
    h->L.mat = take(n);
    h->L.flags[0] = take(n);
    h->L.flags[1] = take(n);
    h->L.mats = take((uint64_t)h->n_mat * (ts == 8 ? sizeof(MatConst<double>) : sizeof(MatConst<float>)));
    h->L.pairs = take((uint64_t)h->n_mat * h->n_mat * (ts == 8 ? sizeof(PairConst<double>) : sizeof(PairConst<float>)));
    h->L.objs = take(h->objs.size() * (ts == 8 ? sizeof(BatchObj<double>) : sizeof(BatchObj<float>)));
    h->wg_cap = (int)h->objs.size();
    h->L.wg_start = take(((uint64_t)h->wg_cap + 1) * 4);
    h->L.wg_objs = take((uint64_t)h->objs.size() * 4);
    h->L.scalars = take(256);
    const uint64_t ns = h->contact ? h->surf_cells.size() : 0;
    h->L.contact_F = take(h->contact ? 3 * n * ts : 0);
    h->L.surf_cells = take(ns * 4);
    h->L.surf_obj = take(ns * 4);
    h->L.surf_ijk = take(ns * 8);
    h->L.obj_origin = take(h->origins.size() * 8);
    h->L.cand = take(ns * (uint64_t)h->cand_cap * 4);
    h->L.cand_n = take(ns * 4);
    h->L.keys = take(ns * 4);
    h->L.gc = take(ns * 8);
    h->L.sorted = take(ns * 4);
    h->L.sgc = take(ns * 8);
    h->L.sijk = take(ns * 8);
    h->L.sobj = take(ns * 4);
    h->L.su = take(3 * ns * ts);
    h->L.bstart = take(h->contact ? ((uint64_t)h->table_size + 1) * 4 : 0);
    h->L.bfill = take(h->contact ? (uint64_t)h->table_size * 4 : 0);
    h->L.block_sum = take(h->contact ? (uint64_t)scan_blocks(h->table_size) * 4 : 0);
    h->L.total = off;
}

static CollideArgs batch_collide(vx_batch_sim *h) {
    CollideArgs c{};
    char *ws = h->ws;
    Scalars *sc = (Scalars *)(ws + h->L.scalars);
    c.surf_cells = (const int *)(ws + h->L.surf_cells);
    c.surf_obj = (const int *)(ws + h->L.surf_obj);
    c.surf_ijk = (const long long *)(ws + h->L.surf_ijk);
    c.obj_origin = (const double *)(ws + h->L.obj_origin);
    c.n_surf = (int)h->surf_cells.size();
    c.cap = h->cand_cap;
    c.cand = (int *)(ws + h->L.cand);
    c.cand_n = (int *)(ws + h->L.cand_n);
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
    return c;
}

// Longest-processing-time packing: biggest objects first, each to the
// workgroup with the least work so far (work = cells, as every cell of an
// object's tiles is visited each step).
static void lpt(const vx_batch_sim *h, int n_wg, std::vector<int> &start, std::vector<int> &order) {
    std::vector<int> ids(h->objs.size());
    std::iota(ids.begin(), ids.end(), 0);
    auto work = [&](int i) { const ObjHost &o = h->objs[i]; return (long long)o.nx * o.ny * o.nz; };
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return work(a) > work(b); });
    using P = std::pair<long long, int>;
    std::priority_queue<P, std::vector<P>, std::greater<P>> q;
    for (int w = 0; w < n_wg; ++w) q.push({0, w});
    std::vector<std::vector<int>> lists(n_wg);
    for (int i : ids) {
        P top = q.top();
        q.pop();
        lists[top.second].push_back(i);
        q.push({top.first + work(i), top.second});
    }
    start.assign(n_wg + 1, 0);
    order.clear();
    for (int w = 0; w < n_wg; ++w) {
        start[w] = (int)order.size();
        order.insert(order.end(), lists[w].begin(), lists[w].end());
    }
    start[n_wg] = (int)order.size();
}

// The object table (offsets, dimensions, tiles, timesteps); waits for the copy.
template <typename T>
static int upload_objs(vx_batch_sim *h) {
    std::vector<BatchObj<T>> ob(h->objs.size());
    for (size_t i = 0; i < ob.size(); ++i) {
        const ObjHost &o = h->objs[i];
        ob[i].off = (unsigned)o.off; ob[i].nx = o.nx; ob[i].ny = o.ny; ob[i].nz = o.nz;
        ob[i].tx = o.tx; ob[i].ty = o.ty; ob[i].dt = (T)o.dt; ob[i].origin_z = (T)o.origin_z;
    }
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.objs, ob.data(), ob.size() * sizeof(BatchObj<T>), hipMemcpyHostToDevice,
                              h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    return VX_OK;
}

// Puts a tile rule in force; the object table on the device follows once bound.
static int apply_tile_rule(vx_batch_sim *h, int rule) {
    h->tile_rule = rule;
    for (ObjHost &o : h->objs) {
        o.tx = o.tile[rule][0];
        o.ty = o.tile[rule][1];
    }
    if (!h->bound) return VX_OK;
    return h->precision == 64 ? upload_objs<double>(h) : upload_objs<float>(h);
}

template <typename T>
static int upload_all(vx_batch_sim *h) {
    hipStream_t s = h->stream;
    std::vector<MatConst<T>> mc;
    std::vector<PairConst<T>> pc;
    pack_tables<T>(h, mc, pc);
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.mats, mc.data(), mc.size() * sizeof(MatConst<T>), hipMemcpyHostToDevice, s));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.pairs, pc.data(), pc.size() * sizeof(PairConst<T>), hipMemcpyHostToDevice, s));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.mat, h->grid.data(), h->total, hipMemcpyHostToDevice, s));
    std::vector<uint8_t> fl(h->total, 0);
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.flags[0], fl.data(), h->total, hipMemcpyHostToDevice, s));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.flags[1], fl.data(), h->total, hipMemcpyHostToDevice, s));
    const int ro = upload_objs<T>(h);
    if (ro != VX_OK) return ro;
    // rest state: zero everywhere except the quaternion w
    std::vector<T> st((size_t)N_WORDS * h->total, T(0));
    std::fill(st.begin() + (size_t)W_QW * h->total, st.begin() + (size_t)(W_QW + 1) * h->total, T(1));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[0], st.data(), st.size() * sizeof(T), hipMemcpyHostToDevice, s));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[1], st.data(), st.size() * sizeof(T), hipMemcpyHostToDevice, s));
    std::vector<unsigned char> sc(256, 0);
    if (h->contact) {
        Scalars first{};
        first.rebuild_flag = 1u;   // candidates are built before the first step
        first.threshold = 2.0 * h->p.voxel_size - h->cmax;
        first.every = 0u;
        std::memcpy(sc.data(), &first, sizeof(first));
        const size_t ns = h->surf_cells.size();
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_cells, h->surf_cells.data(), ns * 4, hipMemcpyHostToDevice, s));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_obj, h->surf_obj.data(), ns * 4, hipMemcpyHostToDevice, s));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.surf_ijk, h->surf_ijk.data(), ns * 8, hipMemcpyHostToDevice, s));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.obj_origin, h->origins.data(), h->origins.size() * 8,
                                  hipMemcpyHostToDevice, s));
        std::vector<int> zeros(std::max<size_t>(ns, (size_t)h->table_size), 0);
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.cand_n, zeros.data(), ns * 4, hipMemcpyHostToDevice, s));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.bfill, zeros.data(), (size_t)h->table_size * 4, hipMemcpyHostToDevice, s));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.block_sum, zeros.data(), (size_t)scan_blocks(h->table_size) * 4,
                                  hipMemcpyHostToDevice, s));
        std::vector<T> cf((size_t)3 * h->total, T(0));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.contact_F, cf.data(), cf.size() * sizeof(T), hipMemcpyHostToDevice, s));
    }
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.scalars, sc.data(), 256, hipMemcpyHostToDevice, s));
    BHIP_OK(h, hipStreamSynchronize(s));
    return VX_OK;
}

template <typename T>
static int run(vx_batch_sim *h, int64_t n) {
    const int n_wg = h->n_wg > 0 ? h->n_wg : default_wg(h);
    std::vector<int> start, order;
    lpt(h, n_wg, start, order);
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.wg_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, h->stream));
    BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.wg_objs, order.data(), order.size() * 4, hipMemcpyHostToDevice, h->stream));
    Scalars *sc = (Scalars *)(h->ws + h->L.scalars);
    BatchArgs<T> b{};
    StepArgs<T> &a = b.base;
    a.stride = h->total;
    a.mat = (const uint8_t *)(h->ws + h->L.mat);
    a.mats = (const MatConst<T> *)(h->ws + h->L.mats);
    a.pairs = (const PairConst<T> *)(h->ws + h->L.pairs);
    a.n_mat = h->n_mat;
    a.l = (T)h->p.voxel_size;
    a.gravity = (T)h->p.gravity;
    a.floor_on = h->p.floor_on;
    a.track_vmax = h->contact ? 1 : 0;
    a.n_forced = 0;
    a.err_flag = &sc->err_flag;
    a.vmax_bits = &sc->vmax_bits;
    a.contact_F = h->contact ? (const T *)(h->ws + h->L.contact_F) : nullptr;
    b.state[0] = (T *)(h->ws + h->L.state[0]);
    b.state[1] = (T *)(h->ws + h->L.state[1]);
    b.flags[0] = (uint8_t *)(h->ws + h->L.flags[0]);
    b.flags[1] = (uint8_t *)(h->ws + h->L.flags[1]);
    b.objs = (const BatchObj<T> *)(h->ws + h->L.objs);
    b.wg_start = (const int *)(h->ws + h->L.wg_start);
    b.wg_objs = (const int *)(h->ws + h->L.wg_objs);
    b.temp_amp = h->p.temp_amp;
    b.temp_freq = h->p.temp_freq;
    b.temp_phase = h->p.temp_phase;
    if (h->contact) {
        // one step per launch: the collision chain and the contact forces
        // read every object's state at t_n, then the batch kernel steps all
        // objects, then the motion bookkeeping
        const CollideArgs c = batch_collide(h);
        for (int64_t i = 0; i < n; ++i) {
            StepArgs<T> ca = a;   // the lattice view the collision kernels take
            ca.s_in = b.state[h->cur];
            ca.flags = b.flags[h->cur];
            ca.dt = (T)h->dt;
            const double wt = 2.0 * kPi * h->p.temp_freq * ((double)h->step * h->dt);
            ca.dT_global = (T)(h->p.temp_amp * std::sin(wt + h->p.temp_phase));
            ca.wt = wt;
            ca.wt_red = (T)std::fmod(wt, 2.0 * kPi);
            BHIP_OK(h, launch_rebuild<T>(ca, c, h->stream));
            BHIP_OK(h, launch_contact<T>(ca, c, (T *)(h->ws + h->L.contact_F), h->stream));
            b.steps = 1;
            b.cur0 = h->cur;
            b.step0 = h->step;
            BHIP_OK(h, launch_batch<T>(b, n_wg, h->stream));
            BHIP_OK(h, launch_motion_update<T>(ca, c, h->stream));
            h->cur = 1 - h->cur;
            h->step += 1;
        }
    } else {
        int64_t left = n;
        while (left > 0) {
            const int k = (int)std::min<int64_t>(left, h->max_steps_per_launch);
            b.steps = k;
            b.cur0 = h->cur;
            b.step0 = h->step;
            BHIP_OK(h, launch_batch<T>(b, n_wg, h->stream));
            h->cur = (h->cur + k) & 1;
            h->step += k;
            left -= k;
        }
    }
    Scalars st;
    BHIP_OK(h, hipMemcpyAsync(&st, h->ws + h->L.scalars, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    if (st.err_flag) return bfail(h, VX_EUNSTABLE, "non-finite value in a batched object's state");
    if (st.overflow) return bfail(h, VX_EOVERFLOW, "collision candidate list overflow (raise contact_cap)");
    return VX_OK;
}

template <typename T>
static int read_obj(vx_batch_sim *h, int obj, double *u, double *q, double *vel, double *omega) {
    const ObjHost &o = h->objs[obj];
    const long long nc = (long long)o.nx * o.ny * o.nz;
    std::vector<T> w((size_t)N_WORDS * nc);
    for (int k = 0; k < N_WORDS; ++k)
        BHIP_OK(h, hipMemcpyAsync(w.data() + (size_t)k * nc,
                                  h->ws + h->L.state[h->cur] + ((size_t)k * h->total + o.off) * sizeof(T),
                                  nc * sizeof(T), hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    const double l = h->p.voxel_size;
    for (long long c = 0; c < nc; ++c) {
        const int m = h->grid[o.off + c];
        const double mass = m ? h->pal[m].rho * l * l * l : 1.0, I = mass * l * l / 6.0;
        for (int k = 0; k < 3; ++k) {
            if (u) u[3 * c + k] = m ? (double)w[(size_t)(W_UX + k) * nc + c] : 0.0;
            if (vel) vel[3 * c + k] = m ? (double)w[(size_t)(W_PX + k) * nc + c] / mass : 0.0;
            if (omega) omega[3 * c + k] = m ? (double)w[(size_t)(W_LX + k) * nc + c] / I : 0.0;
        }
        if (q)
            for (int k = 0; k < 4; ++k) q[4 * c + k] = m ? (double)w[(size_t)(W_QW + k) * nc + c] : (k == 0 ? 1.0 : 0.0);
    }
    return VX_OK;
}

template <typename T>
static int write_obj(vx_batch_sim *h, int obj, const double *u, const double *q, const double *vel,
                     const double *omega) {
    const ObjHost &o = h->objs[obj];
    const long long nc = (long long)o.nx * o.ny * o.nz;
    std::vector<T> w((size_t)N_WORDS * nc);
    for (int k = 0; k < N_WORDS; ++k)
        BHIP_OK(h, hipMemcpyAsync(w.data() + (size_t)k * nc,
                                  h->ws + h->L.state[h->cur] + ((size_t)k * h->total + o.off) * sizeof(T),
                                  nc * sizeof(T), hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    const double l = h->p.voxel_size;
    for (long long c = 0; c < nc; ++c) {
        const int m = h->grid[o.off + c];
        if (!m) continue;
        const double mass = h->pal[m].rho * l * l * l, I = mass * l * l / 6.0;
        for (int k = 0; k < 3; ++k) {
            if (u) w[(size_t)(W_UX + k) * nc + c] = (T)u[3 * c + k];
            if (vel) w[(size_t)(W_PX + k) * nc + c] = (T)(mass * vel[3 * c + k]);
            if (omega) w[(size_t)(W_LX + k) * nc + c] = (T)(I * omega[3 * c + k]);
        }
        if (q)
            for (int k = 0; k < 4; ++k) w[(size_t)(W_QW + k) * nc + c] = (T)q[4 * c + k];
    }
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < N_WORDS; ++k)
            BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[b] + ((size_t)k * h->total + o.off) * sizeof(T),
                                      w.data() + (size_t)k * nc, nc * sizeof(T), hipMemcpyHostToDevice, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    return VX_OK;
}

extern "C" {

int vx_batch_create(const vx_object *objs, int32_t n_obj, const vx_material *palette, int32_t n_mat,
                    const vx_params *params, int32_t precision, void *stream, vx_batch *out) {
    VX_TRY
    if (!out) return VX_EINVAL;
    *out = nullptr;
    if (!objs || n_obj <= 0 || !palette || n_mat < 1 || n_mat > kFusedMaxMat || !params) return VX_EINVAL;
    if (precision != 32 && precision != 64) return VX_EINVAL;
    const vx_params &p = *params;
    if (!(p.voxel_size > 0.0) || !(p.gravity >= 0.0) || !(p.zeta_bond >= 0.0) || !(p.zeta_slow >= 0.0) ||
        !(p.zeta_col >= 0.0) || !(p.dt_scale >= 0.0) || p.dt_scale > 1.0 || p.reserved != 0 ||
        (p.self_collision_on != 0 && p.self_collision_on != 1) || p.contact_cap < 0 || p.contact_cap > kMaxContactCap)
        return VX_EINVAL;
    for (int i = 1; i < n_mat; ++i) {
        const vx_material &m = palette[i];
        if (!(m.E > 0.0) || !(m.rho > 0.0) || !(m.nu > -1.0 && m.nu < 0.5) || !(m.mu_s >= 0.0) || !(m.mu_d >= 0.0) ||
            !std::isfinite(m.cte))
            return VX_EINVAL;
    }
    std::unique_ptr<vx_batch_sim> owner(new vx_batch_sim());
    vx_batch_sim *h = owner.get();
    h->precision = precision;
    h->tsize = precision == 64 ? 8 : 4;
    h->stream = (hipStream_t)stream;
    h->p = p;
    if (h->p.dt_scale == 0.0) h->p.dt_scale = 1.0;
    h->n_mat = n_mat;
    h->pal.assign(palette, palette + n_mat);
    const double l = p.voxel_size;
    long long off = 0;
    std::vector<char> used(n_mat, 0);   // materials present in any object
    for (int i = 0; i < n_obj; ++i) {
        const vx_object &o = objs[i];
        if (!o.grid || o.nx <= 0 || o.ny <= 0 || o.nz <= 0 || o.reserved != 0 || !std::isfinite(o.origin[0]) ||
            !std::isfinite(o.origin[1]) || !std::isfinite(o.origin[2])) {
            return VX_EINVAL;
        }
        const long long nc = (long long)o.nx * o.ny * o.nz;
        ObjHost oh{};
        oh.off = off; oh.nx = o.nx; oh.ny = o.ny; oh.nz = o.nz;
        choose_tiles(oh);
        oh.tx = oh.tile[0][0];
        oh.ty = oh.tile[0][1];
        oh.origin_z = o.origin[2];
        // the object's own stable timestep over its bonded material pairs
        std::vector<char> seen((size_t)n_mat * n_mat, 0), seen_vox(n_mat, 0);
        for (int z = 0; z < o.nz; ++z)
            for (int y = 0; y < o.ny; ++y)
                for (int x = 0; x < o.nx; ++x) {
                    const long long c = x + (long long)o.nx * (y + (long long)o.ny * z);
                    const int m = o.grid[c];
                    if (m >= n_mat) return VX_EINVAL;
                    if (!m) continue;
                    ++oh.nvox;
                    seen_vox[m] = 1;
                    const int idx[3] = {x, y, z}, dim[3] = {o.nx, o.ny, o.nz};
                    const long long st[3] = {1, o.nx, (long long)o.nx * o.ny};
                    for (int a = 0; a < 3; ++a) {
                        if (idx[a] + 1 >= dim[a]) continue;
                        const int m2 = o.grid[c + st[a]];
                        if (m2) seen[(size_t)m * n_mat + m2] = 1;
                    }
                }
        for (int m = 1; m < n_mat; ++m) used[m] |= seen_vox[m];
        const double wmax = max_bond_omega(palette, n_mat, l, seen, seen_vox);
        oh.dt = wmax > 0.0 ? h->p.dt_scale / (2.0 * kPi * wmax) : 0.0;
        if (p.self_collision_on) {
            // surface voxels: a face neighbour empty or outside the object
            for (int z = 0; z < o.nz; ++z)
                for (int y = 0; y < o.ny; ++y)
                    for (int x = 0; x < o.nx; ++x) {
                        const long long c = x + (long long)o.nx * (y + (long long)o.ny * z);
                        if (!o.grid[c]) continue;
                        const int idx[3] = {x, y, z}, dim[3] = {o.nx, o.ny, o.nz};
                        const long long st[3] = {1, o.nx, (long long)o.nx * o.ny};
                        bool surf = false;
                        for (int a = 0; a < 3 && !surf; ++a)
                            for (int d = -1; d <= 1 && !surf; d += 2) {
                                const int k = idx[a] + d;
                                surf = k < 0 || k >= dim[a] || !o.grid[c + d * st[a]];
                            }
                        if (!surf) continue;
                        if (off + c > INT32_MAX) return VX_EINVAL;
                        h->surf_cells.push_back((int)(off + c));
                        h->surf_obj.push_back(i);
                        h->surf_ijk.push_back(pack_ijk(x, y, z));
                    }
            h->origins.insert(h->origins.end(), o.origin, o.origin + 3);
        }
        h->grid.insert(h->grid.end(), o.grid, o.grid + nc);
        h->nvox += oh.nvox;
        h->objs.push_back(oh);
        off += nc;
    }
    h->total = off;
    if (!fused_state_fits(h->total, h->tsize)) return VX_EINVAL;
    if (p.self_collision_on) {
        // one world: the smallest of the objects' stable timesteps for all,
        // and the largest contact size the global signal can produce
        h->contact = true;
        double dt = 0.0;
        for (const ObjHost &o : h->objs)
            if (o.dt > 0.0 && (dt == 0.0 || o.dt < dt)) dt = o.dt;
        h->dt = dt;
        for (ObjHost &o : h->objs) o.dt = dt;
        double cmax = l;
        for (int m = 1; m < n_mat; ++m)
            if (used[m]) cmax = std::max(cmax, l * (1.0 + std::fabs(palette[m].cte * p.temp_amp)));
        h->cmax = cmax;
        h->cand_cap = p.contact_cap > 0 ? p.contact_cap : 32;
        int ts = 1;
        while (ts < 2 * (int)std::max<size_t>(h->surf_cells.size(), 1)) ts <<= 1;
        h->table_size = ts;
    }
    layout(h);
    *out = owner.release();
    return VX_OK;
    VX_CATCH(nullptr)
}

int vx_batch_workspace_bytes(vx_batch h, uint64_t *bytes) {
    VX_TRY
    if (!h || !bytes) return VX_EINVAL;
    *bytes = h->L.total;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_bind_workspace(vx_batch h, void *device_ptr, uint64_t bytes) {
    VX_TRY
    if (!h) return VX_EINVAL;
    if (h->bound) return bfail(h, VX_ESTATE, "workspace already bound");
    if (!device_ptr || bytes < h->L.total) return bfail(h, VX_EINVAL, "workspace too small");
    if (((uintptr_t)device_ptr) % kAlign) return bfail(h, VX_EINVAL, "workspace not 256-byte aligned");
    h->ws = (char *)device_ptr;
    h->bound = true;
    const int r = h->precision == 64 ? upload_all<double>(h) : upload_all<float>(h);
    if (r != VX_OK) h->bound = false;
    return r;
    VX_CATCH(h)
}

int vx_batch_step(vx_batch h, int64_t n) {
    VX_TRY
    if (!h || n < 0) return VX_EINVAL;
    if (!h->bound) return bfail(h, VX_ESTATE, "vx_batch_step before vx_batch_bind_workspace");
    if (n == 0) return VX_OK;
    return h->precision == 64 ? run<double>(h, n) : run<float>(h, n);
    VX_CATCH(h)
}

int vx_batch_read_state(vx_batch h, int32_t obj, double *u, double *q, double *vel, double *omega) {
    VX_TRY
    if (!h || obj < 0 || obj >= (int)h->objs.size()) return VX_EINVAL;
    if (!h->bound) return bfail(h, VX_ESTATE, "read before bind");
    return h->precision == 64 ? read_obj<double>(h, obj, u, q, vel, omega) : read_obj<float>(h, obj, u, q, vel, omega);
    VX_CATCH(h)
}

int vx_batch_write_state(vx_batch h, int32_t obj, const double *u, const double *q, const double *vel,
                         const double *omega) {
    VX_TRY
    if (!h || obj < 0 || obj >= (int)h->objs.size()) return VX_EINVAL;
    if (!h->bound) return bfail(h, VX_ESTATE, "write before bind");
    return h->precision == 64 ? write_obj<double>(h, obj, u, q, vel, omega)
                              : write_obj<float>(h, obj, u, q, vel, omega);
    VX_CATCH(h)
}

int vx_batch_get_dt(vx_batch h, int32_t obj, double *dt) {
    VX_TRY
    if (!h || !dt || obj < 0 || obj >= (int)h->objs.size()) return VX_EINVAL;
    *dt = h->objs[obj].dt;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_counters(vx_batch h, int64_t out[4]) {
    VX_TRY
    if (!h || !out) return VX_EINVAL;
    out[0] = h->step;
    out[1] = (int64_t)h->objs.size();
    out[2] = h->total;
    out[3] = h->nvox;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_candidates(vx_batch h, int32_t *obj_a, int32_t *cell_a, int32_t *obj_b, int32_t *cell_b,
                        int32_t max_pairs, int32_t *n_pairs) {
    VX_TRY
    if (!h || !n_pairs || max_pairs < 0) return VX_EINVAL;
    *n_pairs = 0;
    if (!h->bound || !h->contact) return VX_OK;
    const size_t ns = h->surf_cells.size();
    std::vector<int> cand(ns * h->cand_cap), cn(ns);
    BHIP_OK(h, hipMemcpyAsync(cand.data(), h->ws + h->L.cand, cand.size() * 4, hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipMemcpyAsync(cn.data(), h->ws + h->L.cand_n, cn.size() * 4, hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    int32_t k = 0;
    for (size_t i = 0; i < ns; ++i)
        for (int e = 0; e < cn[i]; ++e) {
            const int j = cand[i * h->cand_cap + e];
            if (j <= (int)i) continue;   // each pair once; list order is object-major
            if (k < max_pairs) {
                const int oi = h->surf_obj[i], oj = h->surf_obj[j];
                if (obj_a) obj_a[k] = oi;
                if (cell_a) cell_a[k] = (int32_t)(h->surf_cells[i] - h->objs[oi].off);
                if (obj_b) obj_b[k] = oj;
                if (cell_b) cell_b[k] = (int32_t)(h->surf_cells[j] - h->objs[oj].off);
            }
            ++k;
        }
    *n_pairs = k;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_contact_counters(vx_batch h, int64_t out[3]) {
    VX_TRY
    if (!h || !out) return VX_EINVAL;
    out[0] = out[1] = 0;
    out[2] = h->contact ? (int64_t)h->surf_cells.size() : 0;
    if (!h->bound || !h->contact) return VX_OK;
    Scalars sc;
    BHIP_OK(h, hipMemcpyAsync(&sc, h->ws + h->L.scalars, sizeof(sc), hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    out[0] = (int64_t)sc.rebuilds;
    out[1] = (int64_t)sc.pair_count;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_set_launch(vx_batch h, int32_t n_workgroups, int32_t max_steps_per_launch) {
    VX_TRY
    if (!h || n_workgroups < 0 || max_steps_per_launch < 0) return VX_EINVAL;
    h->n_wg = std::min<int>(n_workgroups, (int)h->objs.size());
    if (max_steps_per_launch > 0) h->max_steps_per_launch = max_steps_per_launch;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_set_tile_rule(vx_batch h, int32_t rule) {
    VX_TRY
    if (!h || rule < 0 || rule >= kTileRules) return VX_EINVAL;
    return apply_tile_rule(h, rule);
    VX_CATCH(h)
}

int vx_batch_get_tile(vx_batch h, int32_t obj, int32_t out[3]) {
    VX_TRY
    if (!h || !out || obj < 0 || obj >= (int)h->objs.size()) return VX_EINVAL;
    out[0] = h->tile_rule;
    out[1] = h->objs[obj].tx;
    out[2] = h->objs[obj].ty;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_autotune(vx_batch h, int32_t steps, int32_t *n_workgroups) {
    VX_TRY
    if (!h || steps <= 0) return VX_EINVAL;
    if (!h->bound) return bfail(h, VX_ESTATE, "autotune before bind");
    // time each tile rule with candidate workgroup counts on the real
    // objects; the state, the flags, the buffer order, the step count and the
    // status flags are saved and restored around the trial steps, and the
    // tile rule and workgroup count are the fastest pair's, or as before the
    // call on an error
    const size_t bytes = (size_t)N_WORDS * h->total * h->tsize;
    const int cur0 = h->cur;
    const long long step0 = h->step;
    const int wg0 = h->n_wg;
    const int rule0 = h->tile_rule;
    const size_t ns = h->contact ? h->surf_cells.size() : 0;
    std::vector<char> save(bytes), fsave(h->total), ssave(256), csave(ns * h->cand_cap * 4), nsave(ns * 4);
    BHIP_OK(h, hipMemcpyAsync(save.data(), h->ws + h->L.state[cur0], bytes, hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipMemcpyAsync(fsave.data(), h->ws + h->L.flags[cur0], h->total, hipMemcpyDeviceToHost, h->stream));
    BHIP_OK(h, hipMemcpyAsync(ssave.data(), h->ws + h->L.scalars, ssave.size(), hipMemcpyDeviceToHost, h->stream));
    if (ns) {
        BHIP_OK(h, hipMemcpyAsync(csave.data(), h->ws + h->L.cand, csave.size(), hipMemcpyDeviceToHost, h->stream));
        BHIP_OK(h, hipMemcpyAsync(nsave.data(), h->ws + h->L.cand_n, nsave.size(), hipMemcpyDeviceToHost, h->stream));
    }
    BHIP_OK(h, hipStreamSynchronize(h->stream));
    auto restore = [&](int keep_wg) -> int {
        h->n_wg = keep_wg;
        h->cur = cur0;
        h->step = step0;
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.state[cur0], save.data(), bytes, hipMemcpyHostToDevice, h->stream));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.flags[cur0], fsave.data(), h->total, hipMemcpyHostToDevice, h->stream));
        BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.scalars, ssave.data(), ssave.size(), hipMemcpyHostToDevice, h->stream));
        if (ns) {
            BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.cand, csave.data(), csave.size(), hipMemcpyHostToDevice, h->stream));
            BHIP_OK(h, hipMemcpyAsync(h->ws + h->L.cand_n, nsave.data(), nsave.size(), hipMemcpyHostToDevice,
                                      h->stream));
        }
        BHIP_OK(h, hipStreamSynchronize(h->stream));
        return VX_OK;
    };
    const int nobj = (int)h->objs.size();
    const int cands[] = {256, 512, 768, 1024, 1536, 2048, 3072, 4096, INT32_MAX};   // the last: one per object
    hipEvent_t e0, e1;
    BHIP_OK(h, hipEventCreate(&e0));
    BHIP_OK(h, hipEventCreate(&e1));
    float best = 1e30f;
    int best_wg = default_wg(h), best_rule = rule0;
    int rc = VX_OK;
    for (int rule = 0; rule < kTileRules && rc == VX_OK; ++rule) {
        bool same = rule > 0;   // a rule that tiles every object like rule 0 is not timed again
        for (const ObjHost &o : h->objs)
            same = same && o.tile[rule][0] == o.tile[0][0] && o.tile[rule][1] == o.tile[0][1];
        if (same) continue;
        rc = apply_tile_rule(h, rule);
        for (int c : cands) {
            if (rc != VX_OK) break;
            const int nw = std::min(c, nobj);
            h->n_wg = nw;
            float ms = 0.f;
            if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = bfail(h, VX_EDEVICE, "hipEventRecord"); break; }
            rc = h->precision == 64 ? run<double>(h, steps) : run<float>(h, steps);
            if (rc != VX_OK) break;
            if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = bfail(h, VX_EDEVICE, "timing events");
                break;
            }
            if (ms < best) { best = ms; best_wg = nw; best_rule = rule; }
            if (nw == nobj) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != VX_OK) {
        const std::string msg = h->err;
        apply_tile_rule(h, rule0);
        restore(wg0);
        h->err = msg;
        return rc;
    }
    int r = apply_tile_rule(h, best_rule);
    if (r != VX_OK) return r;
    r = restore(best_wg);
    if (r != VX_OK) return r;
    if (n_workgroups) *n_workgroups = best_wg;
    return VX_OK;
    VX_CATCH(h)
}

int vx_batch_destroy(vx_batch h) {
    VX_TRY
    delete h;
    return VX_OK;
    VX_CATCH(nullptr)
}

const char *vx_batch_last_error(vx_batch h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
