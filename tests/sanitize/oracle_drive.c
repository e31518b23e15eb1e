/*
 * Drives every entry point of the oracle over small lattices, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer.  Exits 0 when every
 * call returned what the scenario expects; a sanitizer report aborts first.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vx_oracle.h"

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            fails++;                                                     \
        }                                                                \
    } while (0)

static unsigned long long rng = 0x9E3779B97F4A7C15ull;
static double urand(void) {
    rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static vxo_params base_params(void) {
    vxo_params p;
    memset(&p, 0, sizeof p);
    p.voxel_size = 1e-3;
    p.gravity = 9.81;
    p.zeta_bond = 0.5; p.zeta_slow = 0.002; p.zeta_col = 0.5;
    p.floor_on = 1;
    return p;
}

static void materials(vxo_material *m, int n) {
    memset(m, 0, sizeof(*m) * (size_t)n);
    for (int i = 1; i < n; i++) {
        m[i].E = 1e6 * (double)i; m[i].nu = 0.3; m[i].rho = 1000.0 + 100.0 * i;
        m[i].cte = (i % 2 ? 0.01 : -0.005); m[i].mu_s = 0.8; m[i].mu_d = 0.5;
    }
}

/* every setter, stepping and every read-out on a random heterogeneous lattice */
static void scenario_hetero(int nx, int ny, int nz, int with_channels) {
    vxo_material pal[4];
    materials(pal, 4);
    vxo_params p = base_params();
    p.temp_amp = 10.0; p.temp_freq = 300.0;
    int n = nx * ny * nz;
    uint8_t *g = malloc((size_t)n);
    for (int c = 0; c < n; c++) g[c] = (uint8_t)(urand() < 0.2 ? 0 : 1 + (int)(urand() * 3.0));
    vxo_sim *s = vxo_create(g, nx, ny, nz, pal, 4, &p);
    CHECK(s != NULL);
    if (!s) { free(g); return; }
    int nv = vxo_num_voxels(s), nb = vxo_num_bonds(s);
    CHECK(nv >= 0 && nv <= n && nb >= 0 && nb <= 3 * n);
    double *F = calloc((size_t)n * 6, sizeof(double));
    double *amp = malloc(sizeof(double) * (size_t)n), *ph = malloc(sizeof(double) * (size_t)n);
    uint8_t *fixed = calloc((size_t)n, 1);
    for (int c = 0; c < n; c++) {
        for (int k = 0; k < 6; k++) F[6 * c + k] = 1e-4 * (urand() - 0.5);
        amp[c] = 20.0 * urand(); ph[c] = 6.283 * urand();
        fixed[c] = (uint8_t)(c < nx);
    }
    CHECK(vxo_set_fixed(s, fixed) == VXO_OK);
    CHECK(vxo_set_forces(s, F) == VXO_OK);
    CHECK(vxo_set_actuation(s, amp, ph) == VXO_OK);
    if (with_channels) {
        vxo_channel ch[3] = {{5.0, 200.0, 0.3, 1.0, VXO_WAVE_SINE, 0},
                             {8.0, 150.0, 1.1, 0.0, VXO_WAVE_TRIANGLE, 0},
                             {3.0, 400.0, 0.0, -2.0, VXO_WAVE_SQUARE, 0}};
        int mat_ch[4] = {-1, 0, 1, -1};
        int *cell_ch = malloc(sizeof(int) * (size_t)n);
        for (int c = 0; c < n; c++) cell_ch[c] = (c % 5 == 0) ? 2 : -1;
        CHECK(vxo_set_channels(s, ch, 3, mat_ch, 4, cell_ch) == VXO_OK);
        for (int k = 0; k < 3; k++) CHECK(isfinite(vxo_channel_value(&ch[k], 0.0123)));
        free(cell_ch);
    }
    double *vel = malloc(sizeof(double) * (size_t)n * 3);
    for (int i = 0; i < 3 * n; i++) vel[i] = 1e-3 * (urand() - 0.5);
    CHECK(vxo_set_velocity(s, vel) == VXO_OK);
    CHECK(vxo_dt(s) > 0.0);
    CHECK(vxo_step(s, 150) == VXO_OK);
    CHECK(vxo_time(s) > 0.0);
    double *u = malloc(sizeof(double) * (size_t)n * 3), *q = malloc(sizeof(double) * (size_t)n * 4);
    double *v = malloc(sizeof(double) * (size_t)n * 3), *w = malloc(sizeof(double) * (size_t)n * 3);
    vxo_read_state(s, u, q, v, w);
    for (int i = 0; i < 3 * n; i++) CHECK(isfinite(u[i]) && isfinite(v[i]) && isfinite(w[i]));
    vxo_write_state(s, u, q, v, w);
    uint8_t *st = malloc((size_t)n), *sf = malloc((size_t)n);
    vxo_read_flags(s, st, sf);
    double e[16];
    vxo_energy(s, e);
    for (int k = 0; k < 10; k++) CHECK(isfinite(e[k]));
    int *c1 = malloc(sizeof(int) * (size_t)(nb + 1)), *c2 = malloc(sizeof(int) * (size_t)(nb + 1));
    int *ax = malloc(sizeof(int) * (size_t)(nb + 1));
    double *fm = malloc(sizeof(double) * 9 * (size_t)(nb + 1));
    CHECK(vxo_bond_results(s, c1, c2, ax, fm) == nb);
    CHECK(vxo_step(s, 10) == VXO_OK);
    CHECK(vxo_last_error(s) != NULL);
    free(c1); free(c2); free(ax); free(fm); free(st); free(sf);
    free(u); free(q); free(v); free(w); free(vel); free(fixed); free(amp); free(ph); free(F);
    vxo_destroy(s);
    free(g);
}

/* two cubes driven together with self-collision on: contact, candidate
 * read-out into a short buffer, and the overflow of a one-entry cap */
static void scenario_contact(int cap, double speed, int expect_overflow) {
    vxo_material pal[2];
    materials(pal, 2);
    vxo_params p = base_params();
    p.gravity = 0.0; p.floor_on = 0; p.self_collision_on = 1; p.contact_cap = cap;
    const int nx = 9, ny = 3, nz = 3, n = nx * ny * nz;
    uint8_t g[9 * 3 * 3];
    for (int c = 0; c < n; c++) { int x = c % nx; g[c] = (uint8_t)(x < 3 || x > 5); }
    vxo_sim *s = vxo_create(g, nx, ny, nz, pal, 2, &p);
    CHECK(s != NULL);
    if (!s) return;
    vxo_set_rebuild_every_step(s, 1);
    double vel[9 * 3 * 3 * 3];
    for (int c = 0; c < n; c++) {
        int x = c % nx;
        vel[3 * c] = x < 3 ? speed : -speed; vel[3 * c + 1] = 0.0; vel[3 * c + 2] = 0.0;
    }
    CHECK(vxo_set_velocity(s, vel) == VXO_OK);
    int rc = VXO_OK;
    for (int k = 0; k < 40 && rc == VXO_OK; k++) rc = vxo_step(s, 25);
    if (expect_overflow) {
        CHECK(rc == VXO_EOVERFLOW);
    } else {
        CHECK(rc == VXO_OK);
        int a[4], b[4];
        int np = vxo_candidates(s, a, b, 4);
        CHECK(np >= 0);
        CHECK(vxo_rebuilds(s) > 0);
    }
    double e[16];
    vxo_energy(s, e);
    vxo_destroy(s);
}

/* bond damping far above critical: the step reports instability */
static void scenario_unstable(void) {
    vxo_material pal[2];
    materials(pal, 2);
    vxo_params p = base_params();
    p.zeta_bond = 3.0; p.gravity = 0.0; p.floor_on = 0;
    uint8_t g[27];
    memset(g, 1, sizeof g);
    vxo_sim *s = vxo_create(g, 3, 3, 3, pal, 2, &p);
    CHECK(s != NULL);
    if (!s) return;
    double vel[81];
    for (int i = 0; i < 81; i++) vel[i] = 1e-3 * (urand() - 0.5);
    vxo_set_velocity(s, vel);
    int rc = vxo_step(s, 5000);
    CHECK(rc == VXO_EUNSTABLE);
    CHECK(strlen(vxo_last_error(s)) > 0);
    vxo_destroy(s);
}

/* degenerate inputs: rejected at creation, or an empty lattice that steps */
static void scenario_degenerate(void) {
    vxo_material pal[2];
    materials(pal, 2);
    vxo_params p = base_params();
    uint8_t g[8] = {0};
    CHECK(vxo_create(g, 0, 2, 2, pal, 2, &p) == NULL);
    CHECK(vxo_create(NULL, 2, 2, 2, pal, 2, &p) == NULL);
    uint8_t bad[8] = {0, 0, 0, 7, 0, 0, 0, 0};
    CHECK(vxo_create(bad, 2, 2, 2, pal, 2, &p) == NULL);
    vxo_material neg[2];
    materials(neg, 2);
    neg[1].nu = 0.5;
    uint8_t one = 1;
    CHECK(vxo_create(&one, 1, 1, 1, neg, 2, &p) == NULL);
    vxo_sim *s = vxo_create(g, 2, 2, 2, pal, 2, &p);
    CHECK(s != NULL);
    if (s) {
        CHECK(vxo_num_voxels(s) == 0);
        CHECK(vxo_step(s, 3) == VXO_OK);
        double e[16];
        vxo_energy(s, e);
        vxo_destroy(s);
    }
    s = vxo_create(&one, 1, 1, 1, pal, 2, &p);
    CHECK(s != NULL);
    if (s) {
        CHECK(vxo_num_voxels(s) == 1 && vxo_num_bonds(s) == 0);
        CHECK(vxo_step(s, 100) == VXO_OK);
        vxo_destroy(s);
    }
}

int main(void) {
    scenario_hetero(7, 6, 5, 0);
    scenario_hetero(5, 4, 6, 1);
    scenario_hetero(1, 1, 9, 1);
    scenario_contact(32, 0.5, 0);
    scenario_contact(1, 3.0, 1);
    scenario_unstable();
    scenario_degenerate();
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle drive: all scenarios passed\n");
    return 0;
}
