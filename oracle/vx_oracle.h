/*
 * Oracle of the voxel-lattice step (Hiller & Lipson, arXiv 1212.2845).
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * All arrays are dense over the nx*ny*nz cells, cell index x + nx*(y + ny*z),
 * material 0 = empty.  Units are SI.  Everything is FP64 on one thread.
 */
#ifndef VX_ORACLE_H
#define VX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VXO_OK 0
#define VXO_EUNSTABLE (-3)
#define VXO_EOVERFLOW (-4)

typedef struct {
    double E;     /* elastic modulus, Pa */
    double nu;    /* Poisson ratio */
    double rho;   /* density, kg/m^3 */
    double cte;   /* thermal expansion coefficient, 1/K */
    double mu_s;  /* static friction coefficient with the floor */
    double mu_d;  /* dynamic friction coefficient with the floor */
} vxo_material;

typedef struct {
    double voxel_size;            /* lattice dimension l, m */
    double gravity;               /* m/s^2, acts along -z */
    double zeta_bond, zeta_slow, zeta_col;
    double temp_amp, temp_freq, temp_phase;
    double dt_scale;              /* multiplies the stable timestep; 0 -> 1 */
    double origin[3];             /* world position of the lower corner of cell 0 */
    int32_t floor_on, self_collision_on;
    int32_t contact_cap;          /* candidates per voxel (0 -> 32) */
    int32_t pad;
} vxo_params;

/* Named actuation channel: temperature offset + amp * waveform(theta),
 * theta = 2 pi freq t + phase. */
#define VXO_MAX_CHANNELS 8
#define VXO_WAVE_SINE 0
#define VXO_WAVE_TRIANGLE 1
#define VXO_WAVE_SQUARE 2
typedef struct {
    double amp, freq, phase, offset;
    int32_t waveform;
    int32_t pad;
} vxo_channel;

typedef struct vxo_sim vxo_sim;

vxo_sim *vxo_create(const uint8_t *grid, int nx, int ny, int nz,
                    const vxo_material *pal, int n_mat, const vxo_params *prm);
void vxo_destroy(vxo_sim *s);
int vxo_set_fixed(vxo_sim *s, const uint8_t *mask);
int vxo_set_forces(vxo_sim *s, const double *F);
int vxo_set_actuation(vxo_sim *s, const double *amp, const double *phase);
int vxo_set_velocity(vxo_sim *s, const double *vel);
int vxo_set_channels(vxo_sim *s, const vxo_channel *ch, int n_ch, const int *mat_channel, int n_mat,
                     const int *cell_channel);
double vxo_channel_value(const vxo_channel *c, double t);
int vxo_step(vxo_sim *s, long long n);
void vxo_read_state(const vxo_sim *s, double *u, double *q, double *vel, double *omega);
void vxo_write_state(vxo_sim *s, const double *u, const double *q, const double *vel,
                     const double *omega);
void vxo_read_flags(const vxo_sim *s, uint8_t *is_static, uint8_t *surface);
double vxo_dt(const vxo_sim *s);
double vxo_time(const vxo_sim *s);
int vxo_num_voxels(const vxo_sim *s);
int vxo_num_bonds(const vxo_sim *s);
const char *vxo_last_error(const vxo_sim *s);
void vxo_set_rebuild_every_step(vxo_sim *s, int on);
long long vxo_rebuilds(const vxo_sim *s);
int vxo_candidates(const vxo_sim *s, int *cell_a, int *cell_b, int max_pairs);
void vxo_energy(vxo_sim *s, double *out);
int vxo_bond_results(const vxo_sim *s, int *cell1, int *cell2, int *axis, double *f2m1m2);

#ifdef __cplusplus
}
#endif
#endif
