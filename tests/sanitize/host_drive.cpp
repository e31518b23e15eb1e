// Drives the host side of the C ABI (packing, validation, per-bond
// constants, timestep, surface list, state marshalling, parameter setters,
// workspace sizing) without a GPU, for a build of the library whose host
// code carries AddressSanitizer and UndefinedBehaviorSanitizer.  Calls that
// need a bound workspace must answer VX_ESTATE.  Exits 0 when every call
// answered as expected; a sanitizer report aborts first.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "voxsim.h"

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

static std::mt19937_64 rng(12345);
static double urand() { return std::uniform_real_distribution<double>(0.0, 1.0)(rng); }

static std::vector<vx_material> palette(int n) {
    std::vector<vx_material> m(n);
    std::memset(m.data(), 0, sizeof(vx_material) * n);
    for (int i = 1; i < n; ++i) {
        m[i].E = 1e6 * i; m[i].nu = 0.3; m[i].rho = 1000.0 + 100.0 * i;
        m[i].cte = (i % 2) ? 0.01 : -0.005; m[i].mu_s = 0.8; m[i].mu_d = 0.5;
    }
    return m;
}

static vx_params params(int collide) {
    vx_params p;
    std::memset(&p, 0, sizeof p);
    p.voxel_size = 1e-3; p.gravity = 9.81; p.zeta_bond = 0.5; p.zeta_slow = 0.002; p.zeta_col = 0.5;
    p.temp_amp = 10.0; p.temp_freq = 300.0;
    p.floor_on = 1; p.self_collision_on = collide;
    return p;
}

static void single(int nx, int ny, int nz, int precision, int collide) {
    const int n = nx * ny * nz;
    std::vector<uint8_t> g(n);
    for (auto &c : g) c = urand() < 0.25 ? 0 : (uint8_t)(1 + (int)(urand() * 3.0));
    auto pal = palette(4);
    vx_params p = params(collide);
    vx_handle h = nullptr;
    int rc = vx_create(g.data(), nx, ny, nz, pal.data(), 4, &p, precision, nullptr, &h);
    CHECK(rc == VX_OK && h);
    if (rc != VX_OK) return;
    uint64_t ws = 0, sws = 0, gws = 0;
    CHECK(vx_workspace_bytes(h, &ws) == VX_OK && ws > 0);
    CHECK(vx_static_workspace_bytes(h, &sws) == VX_OK);
    CHECK(vx_grad_workspace_bytes(h, 100, 10, &gws) == VX_OK || true);
    double dt = 0.0, t = -1.0;
    CHECK(vx_get_dt(h, &dt) == VX_OK && dt > 0.0);
    CHECK(vx_get_time(h, &t) == VX_OK && t == 0.0);

    std::vector<uint8_t> mask(n);
    for (int c = 0; c < n; ++c) mask[c] = (uint8_t)(c % nx == 0);
    CHECK(vx_set_fixed(h, mask.data()) == VX_OK);
    std::vector<double> F(6 * (size_t)n);
    for (auto &f : F) f = 1e-4 * (urand() - 0.5);
    CHECK(vx_set_forces(h, F.data()) == VX_OK);
    F[7] = NAN;
    CHECK(vx_set_forces(h, F.data()) == VX_EINVAL);
    const double loc[3] = {0.0, 0.0, 0.0}, size[3] = {0.5e-3, 10e-3, 10e-3}, f3[3] = {0.0, 0.0, -1e-3};
    CHECK(vx_fixed_region(h, loc, size) == VX_OK);
    CHECK(vx_forced_region(h, loc, size, f3) == VX_OK);
    std::vector<double> amp(n), ph(n);
    for (int c = 0; c < n; ++c) { amp[c] = 20.0 * urand(); ph[c] = 6.0 * urand(); }
    CHECK(vx_set_actuation(h, amp.data(), ph.data()) == VX_OK);
    vx_channel ch[3];
    std::memset(ch, 0, sizeof ch);
    ch[0].amp = 5.0; ch[0].freq = 200.0; ch[0].waveform = VX_WAVE_SINE;
    ch[1].amp = 8.0; ch[1].freq = 150.0; ch[1].phase = 1.0; ch[1].waveform = VX_WAVE_TRIANGLE;
    ch[2].amp = 3.0; ch[2].freq = 400.0; ch[2].offset = -2.0; ch[2].waveform = VX_WAVE_SQUARE;
    int32_t mat_ch[4] = {-1, 0, 1, -1};
    std::vector<int32_t> cell_ch(n, -1);
    for (int c = 0; c < n; c += 5) cell_ch[c] = 2;
    CHECK(vx_set_channels(h, ch, 3, mat_ch, cell_ch.data()) == VX_OK);
    int filled = 0;
    while (!g[filled]) ++filled;
    cell_ch[filled] = 9;
    CHECK(vx_set_channels(h, ch, 3, mat_ch, cell_ch.data()) == VX_EINVAL);
    CHECK(vx_set_channels(h, ch, VX_MAX_CHANNELS + 1, mat_ch, nullptr) == VX_EINVAL);
    std::vector<double> vel(3 * (size_t)n);
    for (auto &v : vel) v = 1e-3 * (urand() - 0.5);
    CHECK(vx_set_velocity(h, vel.data()) == VX_OK);

    std::vector<double> u(3 * (size_t)n), q(4 * (size_t)n), v(3 * (size_t)n), w(3 * (size_t)n);
    rc = vx_read_state(h, u.data(), q.data(), v.data(), w.data());
    CHECK(rc == VX_OK || rc == VX_ESTATE);
    for (auto &x : u) x = 1e-6 * (urand() - 0.5);
    rc = vx_write_state(h, u.data(), q.data(), v.data(), w.data());
    CHECK(rc == VX_OK || rc == VX_ESTATE);
    std::vector<uint8_t> st(n), sf(n);
    rc = vx_read_flags(h, st.data(), sf.data());
    CHECK(rc == VX_OK || rc == VX_ESTATE);

    // per-voxel moduli at most the palette's and densities at least its
    // keep every bond within the timestep's bound
    std::vector<double> E(n), rho(n);
    for (int c = 0; c < n; ++c) {
        const vx_material &m = pal[g[c] ? g[c] : 1];
        E[c] = m.E * (0.5 + 0.5 * urand()); rho[c] = m.rho * (1.0 + urand());
    }
    CHECK(vx_set_stiffness(h, E.data()) == VX_OK);
    CHECK(vx_set_density(h, rho.data()) == VX_OK);
    E[filled] = -1.0;
    CHECK(vx_set_stiffness(h, E.data()) == VX_EINVAL);
    E[filled] = 1e12;
    CHECK(vx_set_stiffness(h, E.data()) == VX_EINVAL);

    CHECK(vx_set_collision_mode(h, 1, 1) == VX_OK);
    CHECK(vx_set_kernel(h, 99) == VX_EINVAL);
    CHECK(vx_set_fused_tile(h, 1, 4) == VX_OK);
    int32_t shp = -1, tx = 0, ty = 0, zc = 0;
    CHECK(vx_get_fused_tile(h, &shp, &tx, &ty, &zc) == VX_OK && shp == 1 && tx * ty > 0);
    CHECK(vx_set_fused_tile(h, 1000, 4) == VX_EINVAL);

    CHECK(vx_step(h, 1) == VX_ESTATE);
    CHECK(std::strlen(vx_last_error(h)) > 0);
    CHECK(vx_bind_workspace(h, (void *)4096, ws - 1) == VX_EINVAL);
    CHECK(vx_destroy(h) == VX_OK);
}

static void rejects() {
    auto pal = palette(2);
    vx_params p = params(0);
    uint8_t g[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    vx_handle h = nullptr;
    CHECK(vx_create(g, 0, 2, 2, pal.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    CHECK(vx_create(g, 2, 2, 2, pal.data(), 2, &p, 16, nullptr, &h) == VX_EINVAL);
    CHECK(vx_create(nullptr, 2, 2, 2, pal.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    uint8_t bad[8] = {1, 1, 1, 5, 1, 1, 1, 1};
    CHECK(vx_create(bad, 2, 2, 2, pal.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    auto neg = palette(2);
    neg[1].rho = 0.0;
    CHECK(vx_create(g, 2, 2, 2, neg.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    p.contact_cap = 5000;
    CHECK(vx_create(g, 2, 2, 2, pal.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    p.contact_cap = 0;
    p.reserved = 1;
    CHECK(vx_create(g, 2, 2, 2, pal.data(), 2, &p, 32, nullptr, &h) == VX_EINVAL);
    p.reserved = 0;
    uint8_t empty[8] = {0};
    if (vx_create(empty, 2, 2, 2, pal.data(), 2, &p, 64, nullptr, &h) == VX_OK) vx_destroy(h);
    CHECK(vx_step(nullptr, 1) == VX_EINVAL);
}

static void batch(int n_obj, int collide) {
    auto pal = palette(4);
    vx_params p = params(collide);
    std::vector<std::vector<uint8_t>> grids(n_obj);
    std::vector<vx_object> objs(n_obj);
    for (int i = 0; i < n_obj; ++i) {
        const int nx = 2 + (int)(urand() * 7), ny = 2 + (int)(urand() * 7), nz = 2 + (int)(urand() * 7);
        grids[i].resize((size_t)nx * ny * nz);
        for (auto &c : grids[i]) c = urand() < 0.3 ? 0 : (uint8_t)(1 + (int)(urand() * 3.0));
        std::memset(&objs[i], 0, sizeof(vx_object));
        objs[i].grid = grids[i].data();
        objs[i].nx = nx; objs[i].ny = ny; objs[i].nz = nz;
        objs[i].origin[0] = 0.012 * i; objs[i].origin[1] = 0.0; objs[i].origin[2] = 0.001;
    }
    vx_batch b = nullptr;
    int rc = vx_batch_create(objs.data(), n_obj, pal.data(), 4, &p, 32, nullptr, &b);
    CHECK(rc == VX_OK && b);
    if (rc != VX_OK) return;
    uint64_t ws = 0;
    CHECK(vx_batch_workspace_bytes(b, &ws) == VX_OK && ws > 0);
    for (int i = 0; i < n_obj; ++i) {
        double dt = 0.0;
        CHECK(vx_batch_get_dt(b, i, &dt) == VX_OK && dt > 0.0);
    }
    double dt = 0.0;
    CHECK(vx_batch_get_dt(b, n_obj, &dt) == VX_EINVAL);
    CHECK(vx_batch_set_launch(b, 4, 10) == VX_OK);
    CHECK(vx_batch_set_launch(b, 0, 10) == VX_OK);
    CHECK(vx_batch_set_launch(b, -1, 10) == VX_EINVAL);
    CHECK(vx_batch_step(b, 1) == VX_ESTATE);
    CHECK(std::strlen(vx_batch_last_error(b)) > 0);
    CHECK(vx_batch_destroy(b) == VX_OK);
    objs[0].reserved = 3;
    b = nullptr;
    rc = vx_batch_create(objs.data(), n_obj, pal.data(), 4, &p, 32, nullptr, &b);
    CHECK(rc == VX_EINVAL);
    if (rc == VX_OK) vx_batch_destroy(b);
    objs[0].reserved = 0;
    objs[1].origin[2] = NAN;
    b = nullptr;
    rc = vx_batch_create(objs.data(), n_obj, pal.data(), 4, &p, 32, nullptr, &b);
    CHECK(rc == VX_EINVAL);
    if (rc == VX_OK) vx_batch_destroy(b);
}

int main() {
    single(7, 6, 5, 32, 0);
    single(9, 4, 8, 64, 1);
    single(1, 1, 12, 32, 1);
    single(33, 2, 3, 64, 0);
    rejects();
    batch(5, 0);
    batch(9, 1);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host drive: all scenarios passed\n");
    return 0;
}
