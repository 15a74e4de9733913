/* dcm.h -- C ABI of libdcm.so, the MI355X (gfx950) dynamic cutoff method (DCM) library.
 *
 * The library computes the per-timestep path of the dynamic cutoff method of
 * P. Springer, "A Scalable, Linear-Time Dynamic Cutoff Algorithm for Molecular
 * Simulations of Interfacial Systems" (RWTH Aachen, 2014):
 *   interface detection (Section 4, Fig. 14): binning (Eq. 9-10), smoothing,
 *   two-means density estimate (Eq. 14), labels (Eq. 11-12), removal of small
 *   components (Section 4.2), band-limited distance to the interface
 *   (Eq. 15-19, Section 4.3.2), trilinear interpolation (Alg. 3.1) and the
 *   exponential cutoff function (Eq. 7-8); then Lennard-Jones forces, energy and
 *   virial with per-particle cutoffs (Eq. 4, Alg. 3.2) and velocity-Verlet
 *   integration of Eq. 1-2.
 *
 * Conventions for every entry point:
 *  - Every function returns dcm_status: DCM_OK (0), DCM_PENDING (1) or a negative
 *    error. No exception crosses the ABI. dcm_last_error() returns a thread-local
 *    message for the last non-OK status.
 *  - Pointers named d_* are device (HBM) pointers owned by the caller; h_* are host
 *    pointers. The library never allocates device memory: all device state lives
 *    in a caller-provided workspace (sized by dcm_workspace_bytes) that must stay
 *    valid, untouched, until dcm_destroy.
 *  - Particle arrays are FP64 structure-of-arrays [3][n] (all x, then all y, then
 *    all z) in caller (particle id) order. Internally particles are kept sorted by
 *    cell; outputs are permuted back to caller order.
 *  - Grid arrays have G = Nx*Ny*Nz entries, x fastest: index (k*Ny + j)*Nx + i.
 *  - Work is enqueued on the given stream (a hipStream_t; NULL = default stream)
 *    and the call returns; outputs are valid once the stream reaches that point.
 *    One stream per system; a handle must not be used from two threads at once.
 *  - Units are reduced Lennard-Jones units (sigma, epsilon, mass).
 */
#ifndef DCM_H
#define DCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dcm_status;
enum {
    DCM_OK = 0,
    DCM_PENDING = 1,           /* dcm_poll: request not finished yet                   */
    DCM_E_INVALID = -1,        /* bad argument or parameter set (see dcm_create)       */
    DCM_E_WORKSPACE = -2,      /* workspace missing, misaligned or too small           */
    DCM_E_HIP = -3,            /* a HIP runtime call failed                            */
    DCM_E_BUDGET = -4,         /* serving: request can never fit the memory budget     */
    DCM_E_NONFINITE = -5,      /* non-finite input, or non-finite forces were produced */
    DCM_E_UNKNOWN_TICKET = -6, /* serving: no such request                             */
    DCM_E_NOT_CONVERGED = -7   /* distance iteration hit its sweep limit               */
};

enum { DCM_FP64 = 0, DCM_FP32C = 1 };       /* plain FP64 / FP32 pair math, compensated sums */
enum { DCM_PAIR_I = 0, DCM_PAIR_MAX = 1 };  /* pair (i,j) used iff r < r_c[i] (Alg. 3.2) /
                                               iff r < max(r_c[i], r_c[j]) (symmetric)     */
/* Ensemble of dcm_step: NVE velocity Verlet, or NVT with one Nose-Hoover thermostat
 * (the thesis runs its systems at constant N, V, T, Section 6). */
enum { DCM_NVE = 0, DCM_NOSE_HOOVER = 1 };
/* Shape of the cutoff function between the interface (d = 0) and d = r_c^max: Eq. 7-8's
 * exponential, or the linear ramp r_c^max + (r_c^min - r_c^max) d / r_c^max that Section 3.1
 * and Section 6 (Fig. 34-35) compare it with. */
enum { DCM_CUTOFF_EXP = 0, DCM_CUTOFF_LINEAR = 1 };

typedef void *dcm_stream_t;                 /* a hipStream_t */

/* Method parameters. Defaults in brackets are those of the slab workloads. */
typedef struct {
    double box[3];          /* periodic box edges L_x, L_y, L_z                           */
    double epsilon, sigma;  /* Lennard-Jones parameters of Eq. 4 [1, 1]                   */
    double mass;            /* particle mass [1]                                          */
    double rc_min, rc_max;  /* cutoff range of Eq. 7 [2.5, 6.0]                           */
    double alpha;           /* steepness of Eq. 7 [-0.5]; any non-zero value              */
    double bin;             /* target box edge of Eq. 10 [1.0]: N_k = max(3, round(L_k/bin)) */
    int32_t smooth_passes;  /* passes of the periodic [1,2,1] filter per axis, 0..4 [1]   */
    int32_t min_component;  /* components with fewer boxes are removed (Section 4.2) [27] */
    int32_t detect_every;   /* force evaluation k re-detects the interface iff
                               k % detect_every == 0 [2]; 0 = only at creation            */
    int32_t precision;      /* DCM_FP64 or DCM_FP32C                                      */
    int32_t pair_rule;      /* DCM_PAIR_I or DCM_PAIR_MAX                                 */
    int32_t energy_shift;   /* 1: pair energy V(r) - V(r_c) (forces unchanged) [0]        */
    double dt;              /* velocity-Verlet time step [0.005]                          */
    double temperature;     /* thermostat target T* = k_B T / epsilon (NVT, Section 6) [0.7] */
    double tdamp;           /* thermostat relaxation time tau [0.5]; Q = g T* tau^2          */
    int32_t thermostat;     /* DCM_NVE or DCM_NOSE_HOOVER [DCM_NVE]                       */
    int32_t cutoff_shape;   /* DCM_CUTOFF_EXP or DCM_CUTOFF_LINEAR [DCM_CUTOFF_EXP]       */
    int32_t tail;           /* 1: runtime tail correction of Section 7, Eq. 21-22 [0]; needs
                               DCM_PAIR_I and energy_shift 0. Every force evaluation adds to
                               particle i the pair force, and to e_i half the pair energy
                               (Eq. 22), of the particles beyond r_c[i], for a planar model of
                               the two phases: liquid and vapor densities from the two-means
                               centres (Eq. 14), the plane at the interpolated signed distance
                               to the interface with the normal its gradient. The signed
                               distance needs a second distance solve per detection (the
                               distance of vapor boxes to the liquid), and both bands reach
                               2 r_c^max + max h_k instead of r_c^max + max h_k. The correction
                               is a mean field, not conservative, and adds nothing to the
                               virial.                                                       */
    int32_t vapor_cutoff;   /* 1: dynamic cutoffs in the vapor too, the extension of Eq. 7 that
                               Section 3.1 suggests [0]: particle i gets the cutoff of the
                               larger of its interpolated depth into the liquid and into the
                               vapor, which mirrors Eq. 7 about the interface; a vapor particle
                               r_c^max or more from the liquid gets r_c^min. Needs the second
                               distance solve of the tail correction.                         */
    double ms_nu;           /* > 0: the segmentation of Eq. 13 (two-phase piecewise-constant
                               Mumford-Shah) replaces the plain threshold, with this perimeter
                               weight [0]; densities are the two-means centres, the image is
                               scaled so that the liquid centre is 1 and lengths so that the
                               longest box edge is 1 (the thesis uses nu = 0.005). Solved by
                               ms_iters primal-dual iterations of its convex relaxation from the
                               threshold labels; components are removed afterwards as before. */
    int32_t ms_iters;       /* iterations of that solver, 1..100000 [100]; ignored if ms_nu = 0 */
    int32_t neighbor_list;  /* 1: forces from Verlet neighbour lists (Alg. 3.3) instead of the
                               direct cell traversal [0]. Each list holds the slots within
                               r_c[i] + skin at its build; it is rebuilt (with a re-sort) when
                               twice the largest displacement since the build plus the largest
                               growth of a cutoff exceeds the skin, which the host checks once
                               per step (a stream synchronization). Particles keep their
                               storage order between builds. Needs DCM_PAIR_I; not for the
                               server. The same pairs as the traversal, summed in list order. */
    double skin;            /* list skin r_s > 0 [0.3]; r_c^max + skin must pass the checks
                               that r_c^max does (half the box, stencil boxes)                */
    int32_t list_capacity;  /* slots per list; 0: 1.25 (4/3) pi (r_c^max + skin)^3 (a density
                               of 1.25 sigma^-3) [0]. A longer list fails with DCM_E_INVALID. */
} dcm_params;

/* One thermodynamic record (all FP64 sums in a fixed reduction order).
 * ke = m/2 sum |v|^2; pe = sum_i e_i with e_i = 1/2 sum_j V(r_ij) over the pairs i uses;
 * virial[6] = sum_i 1/2 sum_j r_ij (x) f_ij in the order xx, yy, zz, xy, xz, yz;
 * pairs = number of ordered pairs (i, j) used; step = force-evaluation index k;
 * xi, eta = Nose-Hoover friction and its time integral after the step (0 under NVE): the
 * extended energy ke + pe + Q xi^2 / 2 + g T* eta is conserved (g = 3n - 3). */
typedef struct {
    double ke, pe, virial[6];
    int64_t pairs;
    int64_t step;
    double xi, eta;
} dcm_thermo;

/* Optional outputs of an interface detection. Each member is a caller device pointer
 * or NULL (not wanted). Grid arrays have G entries, particle arrays n (caller order). */
typedef struct {
    uint32_t *count;   /* particles per box, Eq. 9                                       */
    uint32_t *smooth;  /* smoothed counts                                                */
    uint8_t *raw;      /* threshold labels before component removal (0 liquid, 1 vapor)  */
    uint8_t *label;    /* final labels, Eq. 11-12                                        */
    double *dist;      /* box-interface distances, Eq. 5, capped at r_c^max + max h_k
                          (2 r_c^max + max h_k with the tail correction)                 */
    double *rc;        /* per-particle cutoffs r_c[i], Eq. 7                              */
    double *km;        /* [3] vapor centre, liquid centre, threshold (Eq. 14)             */
    int64_t *stats;    /* [6] Lloyd iterations, vapor / liquid components removed,
                          vapor / liquid boxes flipped, distance sweeps                  */
    double *dist_v;    /* distances of the boxes to the liquid (liquid boxes 0), capped like
                          dist; only with tail = 1 or vapor_cutoff = 1, else DCM_E_INVALID */
} dcm_detect_out;

typedef struct dcm_system dcm_system;

/* Library version string (static storage). */
const char *dcm_version(void);

/* Thread-local message describing the last non-OK status of this thread. */
const char *dcm_last_error(void);

/* Grid of Eq. 10 for these parameters: dims = {N_x, N_y, N_z}. Host only.
 * DCM_E_INVALID for a non-positive box or bin. */
dcm_status dcm_grid_dims(const dcm_params *p, int32_t dims[3]);

/* Bytes of device workspace a system of n particles needs (host only, no GPU use).
 * DCM_E_INVALID if the parameter set is rejected (same checks as dcm_create). */
dcm_status dcm_workspace_bytes(const dcm_params *p, int64_t n, size_t *bytes);

/* Create a system from positions d_x and velocities d_v ([3][n], caller order; copied,
 * the caller keeps ownership). d_ws must be 256-byte aligned and hold ws_bytes >=
 * dcm_workspace_bytes. Enqueues: periodic wrap, binning, interface detection and the
 * force evaluation k = 0, so the system is ready for dcm_step. Synchronizes the stream
 * once to validate inputs.
 * DCM_E_INVALID: n < 2 or n >= 2^26 (67,108,864); box edge <= 0; bin <= 0; rc_min <= 0 or
 *   rc_min > rc_max; rc_max >= min(L)/2 (minimum image); N_k < 3; N_k < 2 ceil(rc_max/h_k)
 *   + 2 (a stencil would reach a cell twice); alpha == 0 with rc_min != rc_max
 *   under DCM_CUTOFF_EXP; unknown cutoff_shape;
 *   smooth_passes outside 0..4; min_component < 0; detect_every < 0; dt, mass or sigma
 *   <= 0; epsilon < 0; unknown precision, pair_rule or thermostat; under DCM_NOSE_HOOVER
 *   temperature or tdamp <= 0.
 * DCM_E_WORKSPACE: d_ws NULL, misaligned or too small. DCM_E_NONFINITE: a non-finite
 * coordinate or velocity. DCM_E_HIP: a HIP call failed. *out is set only on DCM_OK. */
dcm_status dcm_create(const dcm_params *p, int64_t n, void *d_ws, size_t ws_bytes,
                      const double *d_x, const double *d_v, dcm_stream_t stream,
                      dcm_system **out);

/* As dcm_create, but resumes a saved state: d_rc [n] holds the cutoffs carried by each
 * particle and step the index k of the force evaluation that state belongs to. The
 * interface is re-detected only if k % detect_every == 0 (Section 3: cutoffs are
 * carried between detections), so a resumed run repeats the original bit for bit. Two
 * options break that: with tail = 1 a state resumed between detections recomputes the
 * distance fields from its own positions (the original kept those of its last detection),
 * and with neighbor_list = 1 the storage order, and with it the order of the force sums,
 * depends on when the lists were last rebuilt. */
dcm_status dcm_create_from_state(const dcm_params *p, int64_t n, void *d_ws, size_t ws_bytes,
                                 const double *d_x, const double *d_v, const double *d_rc,
                                 int64_t step, dcm_stream_t stream, dcm_system **out);

/* Replace every particle's cutoff with d_rc[n] (caller order; each value must lie in
 * [rc_min, rc_max], DCM_E_INVALID is reported by dcm_check otherwise) and recompute the
 * forces of the current state. Used to evaluate Alg. 3.2 on given cutoffs. */
dcm_status dcm_set_cutoffs(dcm_system *s, dcm_stream_t stream, const double *d_rc);

/* Re-run the interface detection of Fig. 14 (Eq. 9-19, Alg. 3.1, Eq. 7) on the current
 * positions, replace the per-particle cutoffs, and write the requested outputs (out may
 * be NULL). Does not recompute forces. */
dcm_status dcm_detect_interface(dcm_system *s, dcm_stream_t stream, const dcm_detect_out *out);

/* Evaluate Alg. 3.2 (Eq. 4 Lennard-Jones, pair used iff r < r_c[i]; only f_i updated) on
 * the current state and cutoffs. Outputs in caller order, each optional (NULL):
 * d_f [3][n] forces, d_e [n] per-particle energy e_i, d_w [6][n] per-particle virial
 * (xx, yy, zz, xy, xz, yz), d_pairs [n] pairs used by each particle, d_th one record
 * (ke of the current velocities). */
dcm_status dcm_compute_forces(dcm_system *s, dcm_stream_t stream, double *d_f, double *d_e,
                              double *d_w, uint32_t *d_pairs, dcm_thermo *d_th);

/* The exact forces of the accuracy measure of Section 6.1.1 (F^exact in Eq. 20): the full
 * Lennard-Jones force and energy of Eq. 4, with no cutoff, summed over every particle j and
 * every periodic image x_j + (a L_x, b L_y, c L_z) closer than R to particle i (the particle's
 * own images included). R may exceed half the box; the lattice sum converges absolutely, so
 * only its part beyond R is missing (of order rho R^-4 for a particle at a planar interface).
 * Evaluated on the current positions; outputs in caller order, each optional (NULL):
 * d_f [3][n], d_e [n] = 1/2 sum_j V(r_ij). Does not change the system's forces or cutoffs.
 * Not part of the per-step path: one lane per particle visits every box within R.
 * DCM_E_INVALID for s NULL, R <= 0 or not finite, or R so large that the kernel would visit
 * more than 4e10 boxes (n (2 ceil(R/h_x) + 3)(2 ceil(R/h_y) + 3)(2 ceil(R/h_z) + 3)). */
dcm_status dcm_exact_forces(dcm_system *s, double R, dcm_stream_t stream, double *d_f, double *d_e);

/* Advance nsteps velocity-Verlet steps (Eq. 1-2): v += dt/(2m) F; x += dt v; wrap;
 * re-bin; re-detect the interface when k % detect_every == 0; forces (Alg. 3.2);
 * v += dt/(2m) F. Under DCM_NOSE_HOOVER each step starts and ends with half a thermostat
 * step: xi += dt/4 G; v *= exp(-xi dt/2); eta += xi dt/2; xi += dt/4 G, with
 * G = (2 ke - g T*)/Q recomputed from the rescaled ke. d_th (optional) receives nsteps
 * records, one per step. nsteps >= 0. */
dcm_status dcm_step(dcm_system *s, int32_t nsteps, dcm_stream_t stream, dcm_thermo *d_th);

/* Nose-Hoover state {xi, eta} (host arrays of 2 doubles), e.g. to checkpoint and resume an
 * NVT run bit for bit with dcm_create_from_state. Both synchronize the stream. A system starts
 * at {0, 0}. DCM_E_INVALID for NULL arguments or non-finite values. */
dcm_status dcm_get_thermostat(dcm_system *s, dcm_stream_t stream, double h_xi_eta[2]);
dcm_status dcm_set_thermostat(dcm_system *s, dcm_stream_t stream, const double h_xi_eta[2]);

/* Copy the current state out (caller order; each pointer optional): d_x, d_v [3][n],
 * d_rc [n]. *h_step (host, optional) receives the force-evaluation index k. */
dcm_status dcm_get_state(dcm_system *s, dcm_stream_t stream, double *d_x, double *d_v,
                         double *d_rc, int64_t *h_step);

/* Synchronize the stream and report sticky device-side conditions raised since the
 * system was created: DCM_E_NONFINITE (a non-finite force), DCM_E_NOT_CONVERGED (the
 * distance sweeps hit their limit), DCM_E_INVALID (smoothed counts beyond the histogram
 * range, or cutoffs outside [rc_min, rc_max]). DCM_OK otherwise. */
dcm_status dcm_check(dcm_system *s, dcm_stream_t stream);

/* Per-stage timing with HIP events on the system's stream (off by default). Stages:
 * 0 kick/drift/key, 1 sort and cell ranges, 2 smoothing, 3 two-means, 4 labels and
 * components, 5 distance (both solves with the tail correction), 6 interpolation and
 * cutoffs, 7 pair forces (the force kernel alone), 8 reductions and the ordering of the force
 * waves for the next launch, 9 tail correction, 10 neighbour-list checks and builds.
 * on: 0 off, 1 every stage, 2 the pair-force stage only (two events per force launch).
 * DCM_E_INVALID for another level. dcm_stage_times synchronizes and returns total
 * milliseconds and launch counts per stage (arrays of DCM_NSTAGES) accumulated since
 * profiling was first switched on. */
#define DCM_NSTAGES 11

/* Number of neighbour-list builds since creation (0 without neighbor_list), host value. */
dcm_status dcm_list_builds(dcm_system *s, int64_t *h_builds);
dcm_status dcm_set_profiling(dcm_system *s, int32_t on);
dcm_status dcm_stage_times(dcm_system *s, double *h_ms, int64_t *h_counts);

/* Release the handle (host memory only; the caller frees the workspace afterwards).
 * Waits for nothing: synchronize the stream first if work is still queued. */
dcm_status dcm_destroy(dcm_system *s);

/* ---- grid stages on caller images (the same kernels the system path runs) ----------
 * dims = {N_x, N_y, N_z}, each >= 3; d_ws of at least dcm_grid_workspace_bytes. */
dcm_status dcm_grid_workspace_bytes(const int32_t dims[3], size_t *bytes);

/* Periodic [1,2,1] smoothing along x, then y, then z, repeated `passes` (0..4) times;
 * integer arithmetic (stands in for the perimeter penalty of Eq. 13). */
dcm_status dcm_grid_smooth(const int32_t dims[3], int32_t passes, const uint32_t *d_in,
                           uint32_t *d_out, void *d_ws, size_t ws_bytes, dcm_stream_t stream);

/* Two-means estimate of the vapor and liquid densities (Eq. 14, Lloyd's iteration from
 * the minimum and maximum): d_km[3] = {rho_v, rho_l, threshold}; d_stats[0] = iterations.
 * A box is liquid iff its value exceeds the threshold. Values must be < 65536. */
dcm_status dcm_grid_two_means(const int32_t dims[3], const uint32_t *d_g, double *d_km,
                              int64_t *d_stats, void *d_ws, size_t ws_bytes, dcm_stream_t stream);

/* Labels of Eq. 11-12 (liquid 0 iff g > d_km[2]) into d_raw, then removal of 6-connected
 * periodic components with fewer than min_component boxes, vapor first, then liquid on the
 * updated image (Section 4.2), into d_label. d_stats[4] (optional): vapor / liquid
 * components removed, vapor / liquid boxes flipped. */
dcm_status dcm_grid_segment(const int32_t dims[3], const uint32_t *d_g, const double *d_km,
                            int32_t min_component, uint8_t *d_raw, uint8_t *d_label,
                            int64_t *d_stats, void *d_ws, size_t ws_bytes, dcm_stream_t stream);

/* dcm_grid_smooth without a workspace, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, hosts that forbid allocation). The
 * intermediate image of the passes lives in a device array of the library (8,388,608 boxes,
 * 32 MiB per device, held until the process ends), so dims must give at most 8,388,608 boxes
 * (DCM_E_INVALID otherwise). Allocates nothing and copies nothing to or from the host. All
 * calls on one device share that array: calls that overlap on one device (other streams, other
 * threads) race. Same result as dcm_grid_smooth, bit for bit. */
dcm_status dcm_grid_smooth_noalloc(const int32_t dims[3], int32_t passes, const uint32_t *d_in,
                                   uint32_t *d_out, dcm_stream_t stream);

/* Distance of liquid boxes (label 0) to the vapor set (label 1): the fixed point of the
 * Godunov upwind update (Eq. 16-19) restricted to values <= cap, all other values set to
 * cap (Section 4.3.2). h = box edges. *d_sweeps (optional, device) = sweeps used. */
dcm_status dcm_grid_distance(const int32_t dims[3], const double h[3], double cap,
                             const uint8_t *d_label, double *d_dist, int64_t *d_sweeps,
                             void *d_ws, size_t ws_bytes, dcm_stream_t stream);


/* ---- serving form -------------------------------------------------------------------
 * A request loop runs many independent systems (each a full system as above) on one GPU.
 * Not a thesis algorithm: it batches the per-step path of Sections 3-4 across systems.
 *
 * A worker thread admits queued requests in arrival order while the front request's device
 * footprint (its dcm_workspace_bytes plus state staging and thermo records) fits the
 * remaining HBM budget and a free range of the pool. Admitted systems stay resident. When the
 * resident set changes, the launches of one detection period are recorded for every system;
 * systems whose periods launch the same kernels in the same order form a group, and each
 * launch position becomes one batched launch over all members' workgroups, captured with the
 * rest of the group's period into one hipGraph. Every batch replays each group's graph, so
 * stepping all resident systems costs the launches of one system. Remaining steps shorter than
 * a period, and systems the argument tables have no room for, run as ordinary launches.
 * Results are copied to host memory on completion.
 * Thread safety: submit/poll/query may be called from any one thread at a time. */
typedef struct dcm_server dcm_server;

typedef struct {
    int64_t submitted, admitted, completed, rejected, queued, running, batches;
    size_t bytes_in_use;
    int64_t groupings;      /* times the resident systems were regrouped (record + capture)  */
    double grouping_ms;     /* host milliseconds spent regrouping                            */
    int64_t grouped_steps;  /* system-periods run by batched graphs                          */
    int64_t eager_steps;    /* system-periods (or tails) run by ordinary launches            */
} dcm_server_stats;

/* d_pool: caller-owned device memory of pool_bytes (256-byte aligned) the server sub-allocates;
 * hbm_budget <= pool_bytes caps the bytes resident at once. The last min(pool_bytes / 16,
 * 16 MiB) of the pool hold the argument tables of the batched launches; systems go in the rest. Work queued on `stream` is waited
 * for first. DCM_E_INVALID for a NULL/misaligned pool or a budget of 0 or above pool_bytes. */
dcm_status dcm_server_create(size_t hbm_budget, void *d_pool, size_t pool_bytes, dcm_stream_t stream,
                             dcm_server **out);

/* Queue one system: parameters as for dcm_create, host arrays h_x, h_v [3][n] (copied; the
 * caller may free them on return), nsteps >= 0 velocity-Verlet steps. *ticket identifies it.
 * DCM_E_BUDGET if its footprint exceeds the budget (it could never be admitted); the checks
 * of dcm_workspace_bytes otherwise. */
dcm_status dcm_submit(dcm_server *sv, const dcm_params *p, int64_t n, const double *h_x, const double *h_v,
                      int32_t nsteps, uint64_t *ticket);

/* DCM_PENDING while the request is queued or running. When it has finished: its status
 * (DCM_OK or the error of its system), and on DCM_OK the final positions and velocities into
 * h_x_out, h_v_out [3][n] (host, optional) and the last step's thermo record into h_last
 * (optional); the ticket is then released. DCM_E_UNKNOWN_TICKET for a ticket never issued or
 * already returned. */
dcm_status dcm_poll(dcm_server *sv, uint64_t ticket, double *h_x_out, double *h_v_out, dcm_thermo *h_last);

/* Counters of the request loop (host copy). */
dcm_status dcm_server_query(dcm_server *sv, dcm_server_stats *st);

/* Stop admitting, let resident systems finish their steps, drop still-queued requests, join
 * the worker and release the handle (the caller frees the pool afterwards). */
dcm_status dcm_server_destroy(dcm_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* DCM_H */
