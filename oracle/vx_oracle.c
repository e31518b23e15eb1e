/*
 * Reference stepper for the voxel-lattice soft-body method of Hiller & Lipson,
 * "Dynamic Simulation of Soft Heterogeneous Objects" (arXiv 1212.2845).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow,
 * single-threaded FP64 implementation written from the paper's text.  It
 * shares no code with the GPU library and is used only by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark.
 *
 * Layout is deliberately naive: an array of voxel structs, an explicit bond
 * list, a per-voxel table of its six bond slots, and O(n^2) brute force for
 * collision candidates.
 *
 * Step, in the paper's order (section "Physics Engine"):
 *   1. actuation: each voxel's thermal strain at t_n            (Volumetric Actuation, Eq. 39-40)
 *   2. every bond: co-rotational beam force and moments         (Simulation elements, Eq. 6-24)
 *      plus bond damping                                        (Damping, Eq. 33-35)
 *   3. every voxel: sum of its bonds in a fixed order           (Eq. 25-26)
 *      + external force, gravity, damping to ground, floor,
 *      voxel-voxel contact, then Coulomb friction               (Collisions, Eq. 36-38)
 *   4. all voxels updated synchronously ("double Euler")        (Integration, Eq. 27-30)
 *   5. collision-horizon bookkeeping                            (Self collision detection)
 *
 * Readings of passages the paper leaves open are marked READING below; each
 * one is also listed in the design notes of the repository.
 *
 * Parity unpinned: the voxel-voxel contact law.  The paper names contact
 * between voxels but gives no force law, so the law below is a reading;
 * the tests pin only its invariants (equal and opposite pair forces,
 * conserved momentum, separation after impact, candidate sets equal to a
 * brute-force search), not its magnitudes.
 */
#include "vx_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------ */
/* small vector / quaternion helpers (plain, unoptimised)              */
/* ------------------------------------------------------------------ */
typedef struct { double x, y, z; } vec3;
typedef struct { double w, x, y, z; } quat;

static vec3 v3(double x, double y, double z) { vec3 r = {x, y, z}; return r; }
static vec3 vadd(vec3 a, vec3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
static vec3 vsub(vec3 a, vec3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
static vec3 vscale(vec3 a, double s) { return v3(a.x * s, a.y * s, a.z * s); }
static double vdot(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static double vnorm(vec3 a) { return sqrt(vdot(a, a)); }
static vec3 vcross(vec3 a, vec3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

static quat qmul(quat a, quat b) {
    quat r;
    r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
    r.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
    r.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
    r.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
    return r;
}
static quat qconj(quat a) { quat r = {a.w, -a.x, -a.y, -a.z}; return r; }
static quat qnormalize(quat a) {
    double n = sqrt(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    quat r = {a.w / n, a.x / n, a.y / n, a.z / n};
    return r;
}
/* rotate v from the body frame of q into the world frame: q v q^-1 */
static vec3 qrotate(quat q, vec3 v) {
    quat p = {0.0, v.x, v.y, v.z};
    quat r = qmul(qmul(q, p), qconj(q));
    return v3(r.x, r.y, r.z);
}
/* rotate v from the world frame into the body frame of q: q^-1 v q */
static vec3 qrotate_inv(quat q, vec3 v) { return qrotate(qconj(q), v); }

/* READING: the angle of voxel 2 relative to voxel 1 is the rotation vector
 * of q1^-1 q2 (axis times angle), taken on the short branch (w >= 0). */
static vec3 qlog_rotvec(quat q) {
    if (q.w < 0.0) { q.w = -q.w; q.x = -q.x; q.y = -q.y; q.z = -q.z; }
    double s = sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
    double k = (s > 0.0) ? 2.0 * atan2(s, q.w) / s : 2.0 / q.w;
    return v3(k * q.x, k * q.y, k * q.z);
}
/* unit quaternion of the rotation by rotation vector r (angle |r|) */
static quat qexp_rotvec(vec3 r) {
    double a = vnorm(r);
    quat q;
    if (a > 0.0) {
        double s = sin(0.5 * a) / a;
        q.w = cos(0.5 * a); q.x = s * r.x; q.y = s * r.y; q.z = s * r.z;
    } else {
        q.w = 1.0; q.x = 0.0; q.y = 0.0; q.z = 0.0;
    }
    return q;
}

/* Axis permutation that carries bond axis a onto +x (a proper rotation:
 * x -> (x,y,z), y -> (y,z,x), z -> (z,x,y)). "to_local" applies it,
 * "to_world" its inverse. */
static vec3 perm_to_local(int a, vec3 v) {
    if (a == 0) return v;
    if (a == 1) return v3(v.y, v.z, v.x);
    return v3(v.z, v.x, v.y);
}
static vec3 perm_to_world(int a, vec3 v) {
    if (a == 0) return v;
    if (a == 1) return v3(v.z, v.x, v.y);
    return v3(v.y, v.z, v.x);
}

/* ------------------------------------------------------------------ */
/* data                                                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int cell;              /* dense cell index x + nx*(y + ny*z) */
    int ix, iy, iz;
    int mat;
    double m, I;           /* mass, rotational inertia */
    double E, G;           /* elastic and shear modulus of this voxel */
    double kv, kphi;       /* translational / rotational stiffness to ground */
    double cte, mu_s, mu_d;
    double amp, phase;     /* actuation amplitude (K) and phase (rad) */
    int chan;              /* actuation channel, or -1 (own / global signal) */
    /* Position D of the paper's state, held as the rest position of the
     * cell plus a displacement U so that bond stretches never subtract two
     * large absolute coordinates (lattice offsets are exact integers times l). */
    vec3 D0, U;
    vec3 P, W;             /* linear momentum, angular momentum */
    quat q;                /* orientation, body -> world */
    vec3 Fext;
    int fixed, is_static, surface;
    int bond_slot[6];      /* bonds at -x,+x,-y,+y,-z,+z ; -1 if none */
    /* per-step scratch */
    double eps;            /* thermal strain at t_n */
    vec3 F, M;
    double Fn;             /* floor normal force at t_n */
    int ncand;
    int *cand;             /* partner voxel ids, ascending */
} voxel;

typedef struct {
    int v1, v2, axis;      /* v1 is the lower voxel along the axis */
    double Ec, Gc;
    double a1, a2, b1, b2, b3;
    double kb, ct, cr;     /* stiffness, damping coefficients */
    /* per-step results: force on voxel 2 and moments on 1 and 2, world frame */
    vec3 F2, M1, M2;
} bond;

struct vxo_sim {
    int nx, ny, nz, ncell;
    double l;
    vxo_params p;
    int nvox, nbond;
    voxel *vox;
    bond *bonds;
    int *cell_to_vox;      /* -1 for empty */
    double dt;
    long long step;
    double t;
    double macc;           /* accumulated maximum motion */
    double cmax;           /* largest voxel size the actuation can produce */
    long long rebuilds;
    int cand_cap;
    int rebuild_every_step;
    int overflow;
    int n_chan;
    vxo_channel chan[VXO_MAX_CHANNELS];
    char err[256];
};

static void set_err(vxo_sim *s, const char *m) {
    strncpy(s->err, m, sizeof(s->err) - 1);
    s->err[sizeof(s->err) - 1] = 0;
}

/* ------------------------------------------------------------------ */
/* setup                                                              */
/* ------------------------------------------------------------------ */
/* Separation D_B - D_A of two voxels: exact lattice offset plus the
 * difference of displacements. */
static vec3 separation(const vxo_sim *s, const voxel *A, const voxel *B) {
    double l = s->l;
    return vadd(v3((B->ix - A->ix) * l, (B->iy - A->iy) * l, (B->iz - A->iz) * l), vsub(B->U, A->U));
}
/* Absolute position D of a voxel. */
static vec3 position(const voxel *V) { return vadd(V->D0, V->U); }

/* Composite of two moduli: springs of half length in series (Eq. 1, 2). */
static double composite(double a, double b) { return 2.0 * a * b / (a + b); }

static void bond_constants(vxo_sim *s, bond *b) {
    const voxel *A = &s->vox[b->v1], *B = &s->vox[b->v2];
    double l = s->l;
    b->Ec = composite(A->E, B->E);
    b->Gc = composite(A->G, B->G);
    /* beam section of a voxel: area l^2, I = l^4/12, J = l^4/6 (Eq. 4, 5);
     * beam length = nominal lattice dimension (READING) */
    double area = l * l, Is = l * l * l * l / 12.0, J = l * l * l * l / 6.0;
    b->a1 = b->Ec * area / l;                 /* Eq. 8  */
    b->a2 = b->Gc * J / l;                    /* Eq. 9  */
    b->b1 = 12.0 * b->Ec * Is / (l * l * l);  /* Eq. 10 */
    b->b2 = 6.0 * b->Ec * Is / (l * l);       /* Eq. 11 */
    b->b3 = 2.0 * b->Ec * Is / l;             /* Eq. 12 */
    /* READING: the bond stiffness used for the timestep and damping is the
     * axial one, a1 (equal to b1 on a cubic lattice). */
    b->kb = b->a1;
    double mmin = A->m < B->m ? A->m : B->m;
    double imin = A->I < B->I ? A->I : B->I;
    /* Eq. 34, 35: c = 2 zeta sqrt(m k); READING: m is the smaller mass of
     * the pair, the rotational stiffness is b3. */
    b->ct = 2.0 * s->p.zeta_bond * sqrt(mmin * b->kb);
    b->cr = 2.0 * s->p.zeta_bond * sqrt(imin * b->b3);
}

vxo_sim *vxo_create(const uint8_t *grid, int nx, int ny, int nz,
                    const vxo_material *pal, int n_mat, const vxo_params *prm) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !grid || !pal || !prm || n_mat < 1) return NULL;
    if (!(prm->voxel_size > 0.0)) return NULL;
    for (int i = 1; i < n_mat; i++)
        if (!(pal[i].E > 0.0) || !(pal[i].rho > 0.0) || !(pal[i].nu > -1.0 && pal[i].nu < 0.5))
            return NULL;
    vxo_sim *s = (vxo_sim *)calloc(1, sizeof(vxo_sim));
    s->nx = nx; s->ny = ny; s->nz = nz; s->ncell = nx * ny * nz;
    s->p = *prm;
    s->l = prm->voxel_size;
    s->cand_cap = prm->contact_cap > 0 ? prm->contact_cap : 32;
    s->cell_to_vox = (int *)malloc(sizeof(int) * (size_t)s->ncell);
    int nv = 0;
    for (int c = 0; c < s->ncell; c++) {
        if (grid[c] >= n_mat) { free(s->cell_to_vox); free(s); return NULL; }
        s->cell_to_vox[c] = grid[c] ? nv++ : -1;
    }
    s->nvox = nv;
    s->vox = (voxel *)calloc((size_t)(nv > 0 ? nv : 1), sizeof(voxel));
    double l = s->l;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int c = x + nx * (y + ny * z);
                int v = s->cell_to_vox[c];
                if (v < 0) continue;
                voxel *V = &s->vox[v];
                const vxo_material *mt = &pal[grid[c]];
                V->cell = c; V->ix = x; V->iy = y; V->iz = z; V->mat = grid[c];
                /* mass of a cubic voxel, and (READING) rotational inertia of a
                 * solid cube about its centre, m (l^2 + l^2) / 12 */
                V->m = mt->rho * l * l * l;
                V->I = V->m * l * l / 6.0;
                V->E = mt->E;
                V->G = mt->E / (2.0 * (1.0 + mt->nu));
                V->kv = mt->E * l;
                V->kphi = mt->E * l * l * l / 6.0;
                V->cte = mt->cte; V->mu_s = mt->mu_s; V->mu_d = mt->mu_d;
                V->amp = prm->temp_amp; V->phase = prm->temp_phase;
                V->chan = -1;
                V->D0 = v3(prm->origin[0] + (x + 0.5) * l, prm->origin[1] + (y + 0.5) * l,
                           prm->origin[2] + (z + 0.5) * l);
                V->U = v3(0.0, 0.0, 0.0);
                V->q.w = 1.0; V->q.x = V->q.y = V->q.z = 0.0;
                for (int k = 0; k < 6; k++) V->bond_slot[k] = -1;
                V->cand = (int *)malloc(sizeof(int) * (size_t)s->cand_cap);
            }
    /* bonds: one per face-adjacent filled pair, voxel 1 the lower one */
    int maxb = 3 * (nv > 0 ? nv : 1);
    s->bonds = (bond *)calloc((size_t)maxb, sizeof(bond));
    int nb = 0;
    for (int v = 0; v < nv; v++) {
        voxel *V = &s->vox[v];
        int idx[3] = {V->ix, V->iy, V->iz};
        int dim[3] = {nx, ny, nz};
        for (int a = 0; a < 3; a++) {
            if (idx[a] + 1 >= dim[a]) continue;
            int j[3] = {idx[0], idx[1], idx[2]};
            j[a] += 1;
            int u = s->cell_to_vox[j[0] + nx * (j[1] + ny * j[2])];
            if (u < 0) continue;
            bond *b = &s->bonds[nb];
            b->v1 = v; b->v2 = u; b->axis = a;
            bond_constants(s, b);
            V->bond_slot[2 * a + 1] = nb;
            s->vox[u].bond_slot[2 * a] = nb;
            nb++;
        }
    }
    s->nbond = nb;
    /* Timestep (Eq. 31, 32): dt = 1 / (2 pi w_max), w = sqrt(k_b / m_min)
     * over all bonds.  READING: with no bond, a voxel's own k_v / m. */
    double wmax = 0.0;
    for (int b = 0; b < nb; b++) {
        double mmin = s->vox[s->bonds[b].v1].m < s->vox[s->bonds[b].v2].m
                          ? s->vox[s->bonds[b].v1].m : s->vox[s->bonds[b].v2].m;
        double w = sqrt(s->bonds[b].kb / mmin);
        if (w > wmax) wmax = w;
    }
    if (nb == 0)
        for (int v = 0; v < nv; v++) {
            double w = sqrt(s->vox[v].kv / s->vox[v].m);
            if (w > wmax) wmax = w;
        }
    double scale = prm->dt_scale > 0.0 ? prm->dt_scale : 1.0;
    s->dt = wmax > 0.0 ? scale / (2.0 * M_PI * wmax) : 0.0;
    /* surface voxels: filled, with an empty or out-of-grid face neighbour */
    for (int v = 0; v < nv; v++) {
        voxel *V = &s->vox[v];
        int surf = 0;
        for (int k = 0; k < 6; k++) if (V->bond_slot[k] < 0) surf = 1;
        V->surface = surf;
    }
    s->cmax = l;
    s->macc = 0.0;
    return s;
}

void vxo_destroy(vxo_sim *s) {
    if (!s) return;
    for (int v = 0; v < s->nvox; v++) free(s->vox[v].cand);
    free(s->vox); free(s->bonds); free(s->cell_to_vox); free(s);
}

/* ------------------------------------------------------------------ */
/* setters / getters (dense per-cell arrays; empty cells ignored)      */
/* ------------------------------------------------------------------ */
int vxo_set_fixed(vxo_sim *s, const uint8_t *mask) {
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        V->fixed = mask[V->cell] ? 1 : 0;
        if (V->fixed) { V->P = v3(0, 0, 0); V->W = v3(0, 0, 0); }
    }
    return 0;
}

int vxo_set_forces(vxo_sim *s, const double *F) {
    for (int v = 0; v < s->nvox; v++) {
        int c = s->vox[v].cell;
        s->vox[v].Fext = v3(F[3 * c], F[3 * c + 1], F[3 * c + 2]);
    }
    return 0;
}

int vxo_set_actuation(vxo_sim *s, const double *amp, const double *phase) {
    for (int v = 0; v < s->nvox; v++) {
        int c = s->vox[v].cell;
        s->vox[v].amp = amp ? amp[c] : s->p.temp_amp;
        s->vox[v].phase = phase ? phase[c] : s->p.temp_phase;
    }
    return 0;
}

/* Named actuation channels (Volumetric Actuation: several independent
 * "temperatures", each driving only some materials).  READING: a channel
 * is a periodic signal of its own amplitude, frequency, phase, offset and
 * waveform; a voxel follows the channel its cell names, else the channel
 * its material names, else its own or the global signal. */
int vxo_set_channels(vxo_sim *s, const vxo_channel *ch, int n_ch, const int *mat_channel, int n_mat,
                     const int *cell_channel) {
    if (n_ch < 0 || n_ch > VXO_MAX_CHANNELS) return -1;
    for (int k = 0; k < n_ch; k++)
        if (ch[k].waveform < VXO_WAVE_SINE || ch[k].waveform > VXO_WAVE_SQUARE) return -1;
    s->n_chan = n_ch;
    for (int k = 0; k < n_ch; k++) s->chan[k] = ch[k];
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        int k = -1;
        if (cell_channel && cell_channel[V->cell] >= 0) k = cell_channel[V->cell];
        else if (mat_channel && V->mat < n_mat) k = mat_channel[V->mat];
        if (k >= n_ch) return -1;
        V->chan = k < 0 ? -1 : k;
    }
    return 0;
}

/* Value of a channel's temperature signal at time t. */
double vxo_channel_value(const vxo_channel *c, double t) {
    double theta = 2.0 * M_PI * c->freq * t + c->phase;
    double w;
    if (c->waveform == VXO_WAVE_SINE) {
        w = sin(theta);
    } else {
        /* position in the period, 0 <= x < 1; both waveforms start at 0
         * (triangle) or +1 (square) and are in phase with the sine */
        double turns = theta / (2.0 * M_PI);
        double x = turns - floor(turns);
        if (c->waveform == VXO_WAVE_TRIANGLE) {
            if (x < 0.25) w = 4.0 * x;
            else if (x < 0.75) w = 2.0 - 4.0 * x;
            else w = 4.0 * x - 4.0;
        } else {
            w = x < 0.5 ? 1.0 : -1.0;
        }
    }
    return c->offset + c->amp * w;
}

int vxo_set_velocity(vxo_sim *s, const double *vel) {
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        if (V->fixed) continue;
        int c = V->cell;
        V->P = vscale(v3(vel[3 * c], vel[3 * c + 1], vel[3 * c + 2]), V->m);
    }
    return 0;
}

void vxo_read_state(const vxo_sim *s, double *u, double *q, double *vel, double *omega) {
    for (int c = 0; c < s->ncell; c++) {
        int v = s->cell_to_vox[c];
        if (v < 0) {
            if (u) { u[3 * c] = u[3 * c + 1] = u[3 * c + 2] = 0.0; }
            if (q) { q[4 * c] = 1.0; q[4 * c + 1] = q[4 * c + 2] = q[4 * c + 3] = 0.0; }
            if (vel) { vel[3 * c] = vel[3 * c + 1] = vel[3 * c + 2] = 0.0; }
            if (omega) { omega[3 * c] = omega[3 * c + 1] = omega[3 * c + 2] = 0.0; }
            continue;
        }
        const voxel *V = &s->vox[v];
        if (u) { u[3 * c] = V->U.x; u[3 * c + 1] = V->U.y; u[3 * c + 2] = V->U.z; }
        if (q) { q[4 * c] = V->q.w; q[4 * c + 1] = V->q.x; q[4 * c + 2] = V->q.y; q[4 * c + 3] = V->q.z; }
        if (vel) { vel[3 * c] = V->P.x / V->m; vel[3 * c + 1] = V->P.y / V->m; vel[3 * c + 2] = V->P.z / V->m; }
        if (omega) { omega[3 * c] = V->W.x / V->I; omega[3 * c + 1] = V->W.y / V->I; omega[3 * c + 2] = V->W.z / V->I; }
    }
}

void vxo_write_state(vxo_sim *s, const double *u, const double *q, const double *vel,
                     const double *omega) {
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        int c = V->cell;
        if (u) V->U = v3(u[3 * c], u[3 * c + 1], u[3 * c + 2]);
        if (q) { V->q.w = q[4 * c]; V->q.x = q[4 * c + 1]; V->q.y = q[4 * c + 2]; V->q.z = q[4 * c + 3]; }
        if (vel) V->P = vscale(v3(vel[3 * c], vel[3 * c + 1], vel[3 * c + 2]), V->m);
        if (omega) V->W = vscale(v3(omega[3 * c], omega[3 * c + 1], omega[3 * c + 2]), V->I);
    }
}

void vxo_read_flags(const vxo_sim *s, uint8_t *is_static, uint8_t *surface) {
    for (int c = 0; c < s->ncell; c++) {
        int v = s->cell_to_vox[c];
        if (is_static) is_static[c] = v >= 0 ? (uint8_t)s->vox[v].is_static : 0;
        if (surface) surface[c] = v >= 0 ? (uint8_t)s->vox[v].surface : 0;
    }
}

double vxo_dt(const vxo_sim *s) { return s->dt; }
double vxo_time(const vxo_sim *s) { return s->t; }
int vxo_num_voxels(const vxo_sim *s) { return s->nvox; }
int vxo_num_bonds(const vxo_sim *s) { return s->nbond; }
const char *vxo_last_error(const vxo_sim *s) { return s->err; }
void vxo_set_rebuild_every_step(vxo_sim *s, int on) { s->rebuild_every_step = on; }
long long vxo_rebuilds(const vxo_sim *s) { return s->rebuilds; }

/* ------------------------------------------------------------------ */
/* forces                                                             */
/* ------------------------------------------------------------------ */
/* Thermal strain of a voxel at time t (Volumetric Actuation).
 * READING: each voxel carries its own temperature signal
 * A sin(2 pi f t + phase); a global signal is the special case of equal A
 * and phase everywhere. */
static double voxel_strain(const vxo_sim *s, const voxel *V, double t) {
    double dT;
    if (V->chan >= 0) dT = vxo_channel_value(&s->chan[V->chan], t);
    else dT = V->amp * sin(2.0 * M_PI * s->p.temp_freq * t + V->phase);
    return V->cte * dT;
}

/* Force and moments of one bond from the state at t_n. */
static void bond_force(vxo_sim *s, bond *b) {
    const voxel *A = &s->vox[b->v1], *B = &s->vox[b->v2];
    int a = b->axis;
    double l = s->l;
    /* Rest length scaled by the mean strain of the two voxels (Eq. 40). */
    double L = l * (1.0 + 0.5 * (A->eps + B->eps));
    /* Transform into the frame of voxel 1, then permute the bond axis onto
     * +x: voxel 1 sits at the origin with zero rotation, so only voxel 2's
     * six displacements remain (text before Eq. 13). */
    vec3 dAB = separation(s, A, B);
    vec3 d = perm_to_local(a, qrotate_inv(A->q, dAB));
    vec3 th = perm_to_local(a, qlog_rotvec(qmul(qconj(A->q), B->q)));
    double X2 = d.x - L, Y2 = d.y, Z2 = d.z;
    /* Nodal forces K u of the 12-DOF beam (Eq. 7) with u1 = 0.  READING:
     * the z-force on node 1 follows the matrix (row 3: -b1 Z2 - b2 thy2);
     * the printed reduced form has the sign of its b2 term flipped, which
     * breaks the element's moment balance. */
    vec3 f2 = v3(b->a1 * X2, b->b1 * Y2 - b->b2 * th.z, b->b1 * Z2 + b->b2 * th.y);
    vec3 m2 = v3(b->a2 * th.x, b->b2 * Z2 + 2.0 * b->b3 * th.y, -b->b2 * Y2 + 2.0 * b->b3 * th.z);
    vec3 m1 = v3(-b->a2 * th.x, b->b2 * Z2 + b->b3 * th.y, -b->b2 * Y2 + b->b3 * th.z);
    /* READING: K u is what must be applied to hold the displacement; the
     * bond acts on the voxels with the opposite sign.  Back to the world
     * frame by the inverse of the same transform. */
    vec3 F2 = vscale(qrotate(A->q, perm_to_world(a, f2)), -1.0);
    vec3 M2 = vscale(qrotate(A->q, perm_to_world(a, m2)), -1.0);
    vec3 M1 = vscale(qrotate(A->q, perm_to_world(a, m1)), -1.0);

    /* Bond damping (Eq. 33-35): relative velocity with the pair's rigid
     * translation and rotation removed. */
    vec3 v1 = vscale(A->P, 1.0 / A->m), v2 = vscale(B->P, 1.0 / B->m);
    vec3 w1 = vscale(A->W, 1.0 / A->I), w2 = vscale(B->W, 1.0 / B->I);
    vec3 Va = vscale(vadd(v1, v2), 0.5);
    vec3 Wa = vscale(vadd(w1, w2), 0.5);
    vec3 r2 = vscale(dAB, 0.5);  /* D2 - Da, Da the mean position of the pair */
    vec3 Vr = vadd(vsub(v2, Va), vcross(r2, Wa));
    vec3 Wr = vsub(w2, Wa);
    F2 = vsub(F2, vscale(Vr, b->ct));
    M2 = vsub(M2, vscale(Wr, b->cr));
    M1 = vadd(M1, vscale(Wr, b->cr));
    b->F2 = F2; b->M1 = M1; b->M2 = M2;
}

/* Brute-force collision candidates (Self collision detection): surface
 * voxel pairs closer than the horizon (READING: centre distance < 2 l),
 * excluding pairs within lattice Manhattan distance 3 of each other. */
static void rebuild_candidates(vxo_sim *s) {
    double H = 2.0 * s->l;
    for (int v = 0; v < s->nvox; v++) s->vox[v].ncand = 0;
    for (int i = 0; i < s->nvox; i++) {
        voxel *A = &s->vox[i];
        if (!A->surface) continue;
        for (int j = i + 1; j < s->nvox; j++) {
            voxel *B = &s->vox[j];
            if (!B->surface) continue;
            int man = abs(A->ix - B->ix) + abs(A->iy - B->iy) + abs(A->iz - B->iz);
            if (man <= 3) continue;
            if (!(vnorm(separation(s, B, A)) < H)) continue;
            /* voxel ids ascend with j, so both lists stay sorted */
            if (A->ncand < s->cand_cap) A->cand[A->ncand++] = j; else s->overflow = 1;
            if (B->ncand < s->cand_cap) B->cand[B->ncand++] = i; else s->overflow = 1;
        }
    }
    s->rebuilds++;
    s->macc = 0.0;
}

int vxo_candidates(const vxo_sim *s, int *cell_a, int *cell_b, int max_pairs) {
    int n = 0;
    for (int v = 0; v < s->nvox; v++)
        for (int k = 0; k < s->vox[v].ncand; k++) {
            int u = s->vox[v].cand[k];
            if (u <= v) continue;
            if (n < max_pairs) { cell_a[n] = s->vox[v].cell; cell_b[n] = s->vox[u].cell; }
            n++;
        }
    return n;
}

/* Coulomb friction with the floor (Eq. 36-38), applied to voxel V whose
 * total force this step is F and whose floor normal force is Fn.
 * READING: F_l is the lateral part of every other force on the voxel, the
 * halt test uses the lateral velocity at t_n, and a halted voxel whose
 * lateral force exceeds the static limit moves off with the dynamic
 * friction force opposing that lateral force. */
static void friction(const vxo_sim *s, voxel *V) {
    if (!(V->Fn > 0.0)) { V->is_static = 0; return; }
    double Fn = V->Fn;
    double Flx = V->F.x, Fly = V->F.y;
    double Fl = sqrt(Flx * Flx + Fly * Fly);
    if (V->is_static) {
        if (Fl <= V->mu_s * Fn) {
            V->F.x = 0.0; V->F.y = 0.0; V->P.x = 0.0; V->P.y = 0.0;
            return;
        }
        V->is_static = 0;
    }
    double vlx = V->P.x / V->m, vly = V->P.y / V->m;
    double vl = sqrt(vlx * vlx + vly * vly);
    if (vl <= V->mu_d * Fn * s->dt / V->m) {
        V->P.x = 0.0; V->P.y = 0.0;
        V->is_static = 1;
        if (Fl <= V->mu_s * Fn) {
            V->F.x = 0.0; V->F.y = 0.0;
        } else {
            V->F.x -= V->mu_d * Fn * Flx / Fl;
            V->F.y -= V->mu_d * Fn * Fly / Fl;
        }
    } else {
        V->F.x -= V->mu_d * Fn * vlx / vl;
        V->F.y -= V->mu_d * Fn * vly / vl;
    }
}

/* ------------------------------------------------------------------ */
/* step                                                               */
/* ------------------------------------------------------------------ */
static int finite3(vec3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

static int step_once(vxo_sim *s) {
    double l = s->l, dt = s->dt;
    double tn = (double)s->step * dt;
    /* 1. actuation strains at t_n */
    for (int v = 0; v < s->nvox; v++) s->vox[v].eps = voxel_strain(s, &s->vox[v], tn);
    /* collision candidates: built before the first step, then either
     * every step (test mode) or when the horizon test below asks for it */
    if (s->p.self_collision_on && (s->rebuilds == 0 || s->rebuild_every_step))
        rebuild_candidates(s);
    /* 2. all bonds from the state at t_n */
    for (int b = 0; b < s->nbond; b++) bond_force(s, &s->bonds[b]);
    /* 3. per-voxel totals, in a fixed order */
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        vec3 F = v3(0, 0, 0), M = v3(0, 0, 0);
        for (int k = 0; k < 6; k++) {
            int bi = V->bond_slot[k];
            if (bi < 0) continue;
            const bond *b = &s->bonds[bi];
            if (k & 1) { /* this voxel is voxel 1 of the bond */
                F = vsub(F, b->F2);
                M = vadd(M, b->M1);
            } else {     /* voxel 2 */
                F = vadd(F, b->F2);
                M = vadd(M, b->M2);
            }
        }
        F = vadd(F, V->Fext);
        /* gravity along -z */
        F.z -= V->m * s->p.gravity;
        /* damping to ground (SetSlowDampZ): READING: the voxel's own
         * stiffness, E l for translation and E l^3 / 6 for rotation */
        vec3 vel = vscale(V->P, 1.0 / V->m), om = vscale(V->W, 1.0 / V->I);
        F = vsub(F, vscale(vel, 2.0 * s->p.zeta_slow * sqrt(V->m * V->kv)));
        M = vsub(M, vscale(om, 2.0 * s->p.zeta_slow * sqrt(V->I * V->kphi)));
        /* floor at z = 0 (Gravity, floor and friction): penetration of the
         * voxel's current (expanded) size, penalty with its own stiffness,
         * normal damping with the collision damping ratio, no adhesion. */
        V->Fn = 0.0;
        if (s->p.floor_on) {
            double size = l * (1.0 + V->eps);
            double pen = 0.5 * size - position(V).z;
            if (pen > 0.0) {
                double cd = 2.0 * s->p.zeta_col * sqrt(V->m * V->kv);
                double Fn = V->kv * pen - cd * vel.z;
                if (Fn < 0.0) Fn = 0.0;
                V->Fn = Fn;
                F.z += Fn;
            }
        }
        /* voxel-voxel contact (READING: the paper gives no law; spheres of
         * the current voxel size, penalty with the pair's composite
         * stiffness, collision damping on the approach speed, no adhesion) */
        if (s->p.self_collision_on && V->ncand > 0) {
            vec3 Fc = v3(0, 0, 0);
            for (int k = 0; k < V->ncand; k++) {
                const voxel *U = &s->vox[V->cand[k]];
                vec3 r = separation(s, U, V);  /* D_v - D_u */
                double dist = vnorm(r);
                double c = 0.5 * l * (1.0 + V->eps) + 0.5 * l * (1.0 + U->eps);
                if (!(dist < c) || !(dist > 0.0)) continue;
                vec3 n = vscale(r, 1.0 / dist);
                double kc = composite(V->E, U->E) * l;
                double mmin = V->m < U->m ? V->m : U->m;
                double cd = 2.0 * s->p.zeta_col * sqrt(mmin * kc);
                vec3 vu = vscale(U->P, 1.0 / U->m);
                double vn = vdot(vsub(vel, vu), n);
                double f = kc * (c - dist) - cd * vn;
                if (f < 0.0) f = 0.0;
                Fc = vadd(Fc, vscale(n, f));
            }
            F = vadd(F, Fc);
        }
        V->F = F; V->M = M;
    }
    /* 4. synchronous update (Eq. 27-30) with friction applied per voxel */
    double vmax = 0.0;
    int ok = 1;
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        if (V->fixed) { V->P = v3(0, 0, 0); V->W = v3(0, 0, 0); continue; }
        if (s->p.floor_on) friction(s, V);
        V->P = vadd(V->P, vscale(V->F, dt));
        vec3 vel = vscale(V->P, 1.0 / V->m);
        V->U = vadd(V->U, vscale(vel, dt));
        V->W = vadd(V->W, vscale(V->M, dt));
        /* READING: the orientation is a unit quaternion advanced by the
         * exact rotation (phi / I) dt, the rotational analogue of Eq. 30 */
        vec3 om = vscale(V->W, 1.0 / V->I);
        V->q = qnormalize(qmul(qexp_rotvec(vscale(om, dt)), V->q));
        double sp = vnorm(vel);
        if (sp > vmax) vmax = sp;
        if (!finite3(V->U) || !finite3(V->P) || !finite3(V->W) || !isfinite(V->q.w)) ok = 0;
    }
    s->step++;
    s->t = (double)s->step * dt;
    /* 5. collision horizon bookkeeping.  READING: the maximum speed times
     * dt is the largest distance any voxel moved; the candidate list must
     * be rebuilt before two voxels outside the horizon can touch, i.e. once
     * twice the accumulated motion reaches the horizon minus the largest
     * contact distance. */
    if (s->p.self_collision_on && !s->rebuild_every_step) {
        s->macc += vmax * dt;
        if (2.0 * s->macc >= 2.0 * l - s->cmax) rebuild_candidates(s);
    }
    if (!ok) { set_err(s, "non-finite state"); return VXO_EUNSTABLE; }
    if (s->overflow) { set_err(s, "collision candidate list overflow"); return VXO_EOVERFLOW; }
    return VXO_OK;
}

int vxo_step(vxo_sim *s, long long n) {
    if (s->p.self_collision_on) {
        /* largest contact size the actuation can produce */
        double cmax = s->l;
        for (int v = 0; v < s->nvox; v++) {
            const voxel *V = &s->vox[v];
            double a = V->chan >= 0 ? fabs(s->chan[V->chan].offset) + fabs(s->chan[V->chan].amp) : fabs(V->amp);
            double sz = s->l * (1.0 + fabs(V->cte) * a);
            if (sz > cmax) cmax = sz;
        }
        s->cmax = cmax;
    }
    for (long long i = 0; i < n; i++) {
        int r = step_once(s);
        if (r != VXO_OK) return r;
    }
    return VXO_OK;
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                        */
/* ------------------------------------------------------------------ */
/* out[0] kinetic energy, out[1] elastic energy of the bonds, out[2]
 * gravitational energy, out[3] floor spring energy, out[4] sum over voxels
 * of v.F + w.M with the undamped conservative forces, out[5] total linear
 * momentum magnitude squared (debug), out[6..8] total linear momentum,
 * out[9..11] total angular momentum about the origin. */
void vxo_energy(vxo_sim *s, double *out) {
    double l = s->l;
    double tn = (double)s->step * s->dt;
    for (int v = 0; v < s->nvox; v++) s->vox[v].eps = voxel_strain(s, &s->vox[v], tn);
    double ke = 0, ue = 0, ug = 0, uf = 0, pw = 0;
    vec3 Ptot = v3(0, 0, 0), Ltot = v3(0, 0, 0);
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        ke += 0.5 * vdot(V->P, V->P) / V->m + 0.5 * vdot(V->W, V->W) / V->I;
        ug += V->m * s->p.gravity * position(V).z;
        V->F = v3(0, 0, 0); V->M = v3(0, 0, 0);
        Ptot = vadd(Ptot, V->P);
        Ltot = vadd(Ltot, vadd(vcross(position(V), V->P), V->W));
    }
    for (int bi = 0; bi < s->nbond; bi++) {
        bond *b = &s->bonds[bi];
        const voxel *A = &s->vox[b->v1], *B = &s->vox[b->v2];
        double L = l * (1.0 + 0.5 * (A->eps + B->eps));
        vec3 d = perm_to_local(b->axis, qrotate_inv(A->q, separation(s, A, B)));
        vec3 th = perm_to_local(b->axis, qlog_rotvec(qmul(qconj(A->q), B->q)));
        double X2 = d.x - L, Y2 = d.y, Z2 = d.z;
        /* 1/2 u2^T K22 u2, K22 the lower-right 6x6 block of Eq. 7 */
        ue += 0.5 * (b->a1 * X2 * X2 + b->b1 * Y2 * Y2 + b->b1 * Z2 * Z2 + b->a2 * th.x * th.x +
                     2.0 * b->b3 * th.y * th.y + 2.0 * b->b3 * th.z * th.z) +
              b->b2 * Z2 * th.y - b->b2 * Y2 * th.z;
        /* conservative (undamped) bond forces for the shadow-energy term */
        double ct = b->ct, cr = b->cr;
        b->ct = 0.0; b->cr = 0.0;
        bond_force(s, b);
        b->ct = ct; b->cr = cr;
        s->vox[b->v1].F = vsub(s->vox[b->v1].F, b->F2);
        s->vox[b->v2].F = vadd(s->vox[b->v2].F, b->F2);
        s->vox[b->v1].M = vadd(s->vox[b->v1].M, b->M1);
        s->vox[b->v2].M = vadd(s->vox[b->v2].M, b->M2);
    }
    for (int v = 0; v < s->nvox; v++) {
        voxel *V = &s->vox[v];
        vec3 F = V->F;
        F.z -= V->m * s->p.gravity;
        if (s->p.floor_on) {
            double pen = 0.5 * l * (1.0 + V->eps) - position(V).z;
            if (pen > 0.0) { uf += 0.5 * V->kv * pen * pen; F.z += V->kv * pen; }
        }
        if (V->fixed) continue;
        pw += vdot(vscale(V->P, 1.0 / V->m), F) + vdot(vscale(V->W, 1.0 / V->I), V->M);
    }
    out[0] = ke; out[1] = ue; out[2] = ug; out[3] = uf; out[4] = pw;
    out[5] = vdot(Ptot, Ptot);
    out[6] = Ptot.x; out[7] = Ptot.y; out[8] = Ptot.z;
    out[9] = Ltot.x; out[10] = Ltot.y; out[11] = Ltot.z;
}

/* Bond results of the last step, for white-box tests: per bond the voxel
 * cells and F2, M1, M2 (world frame). */
int vxo_bond_results(const vxo_sim *s, int *cell1, int *cell2, int *axis, double *f2m1m2) {
    for (int b = 0; b < s->nbond; b++) {
        const bond *B = &s->bonds[b];
        if (cell1) cell1[b] = s->vox[B->v1].cell;
        if (cell2) cell2[b] = s->vox[B->v2].cell;
        if (axis) axis[b] = B->axis;
        if (f2m1m2) {
            double *o = f2m1m2 + 9 * b;
            o[0] = B->F2.x; o[1] = B->F2.y; o[2] = B->F2.z;
            o[3] = B->M1.x; o[4] = B->M1.y; o[5] = B->M1.z;
            o[6] = B->M2.x; o[7] = B->M2.y; o[8] = B->M2.z;
        }
    }
    return s->nbond;
}
