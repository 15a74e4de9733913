/* dcm_oracle.h -- TEST INFRASTRUCTURE, not product code.
 *
 * Plain, slow, single-threaded FP64 reference of the dynamic cutoff method's
 * per-timestep path (P. Springer, "A Scalable, Linear-Time Dynamic Cutoff
 * Algorithm for Molecular Simulations of Interfacial Systems", 2014).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it. It shares no code with the HIP library.
 *
 * Arrays of particle coordinates are [3][n] (all x, then all y, then all z).
 * Grids are [Nz][Ny][Nx] with x fastest (linear index (k*Ny + j)*Nx + i).
 */
#ifndef DCM_ORACLE_H
#define DCM_ORACLE_H
#include <stdint.h>

typedef struct {
    double box[3];
    double epsilon, sigma, mass;
    double rc_min, rc_max, alpha;
    double bin;
    int32_t smooth_passes, min_component, detect_every, pair_rule, energy_shift;
    double dt;
    double temperature, tdamp;   /* Nose-Hoover target T* and relaxation time tau       */
    int32_t thermostat;          /* 0: constant energy, 1: Nose-Hoover (constant T)     */
    int32_t cutoff_shape;        /* 0: exponential (Eq. 7-8), 1: linear ramp            */
    int32_t tail;                /* 1: add the runtime tail correction (Eq. 21-22)      */
    int32_t vapor_cutoff;        /* 1: dynamic cutoffs in the vapor too (Section 3.1)   */
    double ms_nu;                /* > 0: Mumford-Shah segmentation (Eq. 13), its nu     */
    int32_t ms_iters;            /* primal-dual iterations of that segmentation         */
} orc_params;

typedef struct {
    double ke, pe, virial[6];
    int64_t pairs, step;
    double xi, eta;              /* thermostat friction and its time integral           */
} orc_thermo;

/* outputs of one interface detection (every array caller-allocated) */
typedef struct {
    uint32_t *count;   /* [G] particles per box (Eq. 9)                 */
    uint32_t *smooth;  /* [G] smoothed image                            */
    uint8_t  *raw;     /* [G] threshold labels before component removal */
    uint8_t  *label;   /* [G] final labels, 0 liquid / 1 vapor (Eq. 12) */
    double   *dist;    /* [G] box-interface distances (Eq. 5), capped   */
    double   *d;       /* [n] particle-interface distances (Eq. 6)      */
    double   *rc;      /* [n] per-particle cutoffs (Eq. 7)              */
    double    km[3];   /* vapor centre, liquid centre, threshold        */
    int64_t   stats[6];/* lloyd iters, vapor comps removed, liquid comps removed,
                          vapor boxes flipped, liquid boxes flipped, distance rounds */
    double   *dist_v;  /* [G] box-liquid distances (computed when tail or vapor_cutoff is set),
                          capped */
} orc_detect_out;

int     orc_grid(const orc_params *p, int32_t dims[3], double h[3]);
void    orc_wrap(const orc_params *p, int64_t n, double *x);
void    orc_bin(const orc_params *p, int64_t n, const double *x, uint32_t *count, uint32_t *cell);
void    orc_smooth(const int32_t dims[3], int32_t passes, const uint32_t *in, uint32_t *out);
int32_t orc_two_means(int64_t G, const uint32_t *g, double km[3]);
int64_t orc_components(const int32_t dims[3], const uint8_t *s, uint8_t phase,
                       uint32_t *comp, uint32_t *size);
void    orc_segment(const int32_t dims[3], const uint32_t *g, double t, int32_t min_component,
                    uint8_t *raw, uint8_t *label, int64_t stats[4]);
void    orc_ms_solve(const int32_t dims[3], const double *r, const double w[3], int32_t iters,
                     double *u);
void    orc_mumford_shah(const int32_t dims[3], const double h[3], double Lmax, const uint32_t *g,
                         const double km[3], double nu, int32_t iters, uint8_t *raw, double *u_out);
int64_t orc_distance(const int32_t dims[3], const double h[3], double cap, const uint8_t *label,
                     double *dist);
double  orc_godunov(const double a[3], const double h[3]);
double  orc_cutoff(const orc_params *p, double d);
double  orc_interp(const int32_t dims[3], const double h[3], const double *dist, const double xp[3]);
int     orc_detect(const orc_params *p, int64_t n, const double *x, orc_detect_out *out);
void    orc_forces(const orc_params *p, int64_t n, const double *x, const double *rc,
                   int64_t m, const int64_t *subset, int32_t method,
                   double *f, double *e, double *w, int64_t *pairs);
void    orc_forces_images(const orc_params *p, int64_t n, const double *x, double R, int64_t m,
                          const int64_t *subset, double *f, double *e);
void    orc_tail_planar(const orc_params *p, double rc, double delta, double rho_l, double rho_v,
                        double *f_normal, double *du);
double  orc_interp_grad(const int32_t dims[3], const double h[3], const double *D,
                        const double xp[3], double grad[3]);
void    orc_tail(const orc_params *p, const double *dist_l, const double *dist_v,
                 const double km[3], int64_t n, const double *x, const double *rc,
                 double *f, double *du);
int     orc_run(const orc_params *p, int64_t n, double *x, double *v, double *rc, double *f,
                int64_t k0, int32_t nsteps, int32_t method, double nh[2], orc_thermo *th);

#endif
