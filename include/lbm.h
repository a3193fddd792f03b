/*
 * lbm.h -- C-ABI of the MI355X (gfx950) two-fluid colour lattice Boltzmann library.
 *
 * The library advances the colour LBM of McClure, Li, Berrill and Ramstad (arXiv 2007.12266,
 * section "Color Lattice-Boltzmann Model"): two D3Q7 mass-transport LBEs for the component
 * densities N_a and N_b, coupled through the phase indicator phi = (N_a - N_b)/(N_a + N_b), its
 * colour gradient C and the normal n = C/|C| to a D3Q19 MRT momentum LBE that carries the
 * interfacial-tension terms (sigma_ab = 6 alpha) and a constant body force F, over the pore
 * voxels of a labelled rock image whose solid labels carry a wetting affinity phi_s in [-1, 1]
 * (section "Modeling Wetting with Lattice Boltzmann models": cos(theta_eq) = phi_s).
 *
 * Conventions shared by every entry point
 *   - Every call returns lbm_status; LBM_OK == 0. On failure lbm_last_error() returns a
 *     thread-local message describing the last error of the calling thread.
 *   - Dense arrays are nz*ny*nx, C order, x fastest: index = x + nx*(y + ny*z).
 *   - The caller owns every host array it passes; the library copies what it needs before the
 *     call returns. The library owns all device memory of a domain (allocated through the
 *     optional allocator hook, else hipMalloc) and frees it in lbm_domain_destroy.
 *   - Stepping is asynchronous on the domain's HIP stream. Calls that return data to the host
 *     (read_field, reduce, read_history, state_save, step_timed) synchronise that stream.
 *   - A domain handle is not thread-safe: use one domain from one host thread at a time.
 *   - Device pointers are never exposed; every pointer argument below is a host pointer except
 *     where stated (hip_stream is a hipStream_t handle).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_domain lbm_domain; /* opaque; owned by the library */
typedef struct lbm_pool lbm_pool;     /* opaque; owned by the library */

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = 1,      /* invalid argument; nothing was changed                     */
    LBM_ERR_OOM = 2,      /* device allocation failed                                  */
    LBM_ERR_DEVICE = 3,   /* a HIP runtime call failed; the domain should be destroyed  */
    LBM_ERR_UNSTABLE = 4, /* a reduction saw a non-finite value; sticky until state_load */
    LBM_ERR_STATE = 5     /* state buffer does not match this domain                   */
} lbm_status;

/* Storage and arithmetic of the state.
 *   FP64       every value in double, double arithmetic.
 *   FP32_DEV   the D3Q19 populations as float deviations f_q - t_q from the rest equilibrium,
 *              the D3Q7 moment slots, phi and N as float, float arithmetic (the densities summed
 *              in double): 328 bytes per pore voxel and step against 560.
 *   FP32_MIXED the D3Q19 populations as float deviations, the phase field (D3Q7 moment slots,
 *              phi, N) in double, double arithmetic: 408 bytes per pore voxel and step. Rounding
 *              the phase field to float every step is what moves the Darcy flux of a two-phase
 *              state; rounding f moves it about a thousand times less.
 * Reductions and read-back are FP64 in every mode. */
typedef enum { LBM_FP64 = 0, LBM_FP32_DEV = 1, LBM_FP32_MIXED = 2 } lbm_precision;

/* How the kernels find a pore voxel's 18 D3Q19 neighbours. TABLE: an int32 table of 18 entries
 * per pore voxel, read every step (72 bytes per voxel and step). RANK: computed from the voxel's
 * packed coordinate and a per-64-voxel record of the image (pore and solid bitmasks with running
 * indices: about 0.5 byte per image voxel, read through the caches), 4 bytes per voxel and step
 * and 68 bytes less device memory per pore voxel, but slower on MI355X (the lookup adds a
 * dependent load to every gather); needs nx <= 1024 and ny, nz <= 2048. COMPACT: the table's
 * entries as 16-bit codes above per-wave bases (64 consecutive pore voxels share a base per
 * direction) with an 18-bit solid mask: 40 bytes per voxel plus 160 bytes per 64 voxels, the
 * few waves whose targets spread beyond 16 bits keeping int32 entries: about 37 bytes per
 * voxel and step less to read than TABLE, and the fastest of the three on MI355X. AUTO takes
 * COMPACT.
 * Results are bitwise identical. */
typedef enum {
    LBM_NBR_AUTO = 0, LBM_NBR_TABLE = 1, LBM_NBR_RANK = 2, LBM_NBR_COMPACT = 3
} lbm_neighbour_mode;

/* Label kinds (section "Initial conditions and wetting maps": every voxel carries an integer
 * label naming its material). */
typedef enum {
    LBM_LABEL_SOLID = 0,     /* solid; its affinity is the wetting pseudo-phase phi_s       */
    LBM_LABEL_FLUID_A = 1,   /* pore initially filled with fluid a (phi = +1, water)        */
    LBM_LABEL_FLUID_B = 2,   /* pore initially filled with fluid b (phi = -1)               */
    LBM_LABEL_PORE_INIT = 3  /* pore whose initial phi comes from init_phi                  */
} lbm_label_kind;

/* Fields readable with lbm_read_field; all are functions of the stored state after the last
 * completed step (N_a, N_b from the D3Q7 populations; rho = sum f; u = sum f xi + F/2;
 * p = rho/3, the D3Q19 equation of state with cs^2 = 1/3). */
typedef enum {
    LBM_FIELD_NA = 0, LBM_FIELD_NB = 1, LBM_FIELD_PHI = 2, LBM_FIELD_RHO = 3,
    LBM_FIELD_P = 4, LBM_FIELD_UX = 5, LBM_FIELD_UY = 6, LBM_FIELD_UZ = 7
} lbm_field;

/* Optional device-memory hook (e.g. a framework's caching allocator). alloc returns a device
 * pointer of at least `bytes` bytes, 256-byte aligned, or NULL on failure; free releases it. */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} lbm_allocator;

typedef struct {
    int32_t nx, ny, nz;      /* dense image size                                           */
    int32_t periodic[3];     /* per axis; a non-periodic face is a solid wall of            */
                             /* affinity wall_affinity (halfway bounce-back)                */
    double tau_a, tau_b;     /* relaxation times of fluids a and b; nu = (tau - 1/2)/3      */
    double alpha;            /* interfacial-tension parameter: sigma_ab = 6 alpha           */
    double beta;             /* recolouring (interface width) parameter, 0 < beta < 1       */
    double force[3];         /* constant body force per unit volume, lattice units          */
    double wall_affinity;    /* phi_s seen across non-periodic faces                        */
    int32_t bc_z;            /* 0: none; 1: pressure faces at z = 0 (inlet, pure fluid a)   */
                             /* and z = nz-1 (outlet, pure fluid b); needs periodic[2] == 0 */
    int32_t precision;       /* lbm_precision                                               */
    double rho_in, rho_out;  /* imposed densities of the pressure faces (bc_z == 1)         */
    int32_t reduce_every;    /* lbm_step records a reduction every this many steps (0: off) */
    int32_t block_size;      /* threads per workgroup (64, 128 or 256); 0: auto             */
    int32_t neighbour_mode;  /* lbm_neighbour_mode                                        */
    int32_t inlet_mode;      /* with bc_z == 1: 0 imposes rho_in at the inlet; 1 imposes the */
                             /* total flow rate flux_in (the paper's flux condition: every    */
                             /* step the inlet density is the one for which u_z summed over  */
                             /* the inlet plane's pore voxels equals flux_in)                 */
    double flux_in;          /* inlet_mode 1: imposed sum of u_z over the inlet plane         */
    int32_t order_rows;      /* pore numbering: blocks of R rows of y, each block plane by    */
                             /* plane and row by row (neighbours one plane away stay close); */
                             /* 0 = 16 rows; R >= ny = dense order (z, y, x). Results do not */
                             /* depend on it.                                                 */
    int32_t pad_;
    double rho_a, rho_b;     /* densities of fluids a and b. The model is the incompressible  */
                             /* form with unit reference density (the paper runs density     */
                             /* ratio 1), so both must be 1; 0 is read as 1 (a zeroed struct) */
                             /* and any other value is LBM_ERR_ARG                             */
} lbm_params;

/* Reductions over the pore voxels (section "Analysis framework", integral measures, and the
 * total capillary number of the steady-state protocol), accumulated in FP64:
 *   mass_a, mass_b   sum of N_a, N_b;
 *   sw               mean of (1 + phi)/2 over pore voxels (smooth saturation of fluid a);
 *   sw_count         fraction of pore voxels with phi > 0 (volume of the water region);
 *   flux[3]          sum of u over pore voxels / (nx*ny*nz)  (superficial Darcy flux);
 *   flux_a, flux_b   same, weighted by (1 + phi)/2 and (1 - phi)/2;
 *   p_a, p_b         mean p = rho/3 over {phi > 0} and {phi < 0};
 *   ca               (eps_a mu_a |U_a| + eps_b mu_b |U_b|) / (6 alpha) with U = P/M over each
 *                    region (P = sum rho u, M = sum rho), eps = region volume / (nx*ny*nz),
 *                    mu = nu (unit density);
 *   n_pore, step     pore count and the step the reduction describes;
 *   unstable         1 if any N_a, N_b, rho or u was not finite.                              */
typedef struct {
    double mass_a, mass_b, sw, sw_count;
    double flux[3], flux_a[3], flux_b[3];
    double p_a, p_b, ca;
    int64_t n_pore, step;
    int32_t unstable, pad_;
} lbm_reduction;

/* Average device time per launch of each kernel over a lbm_step_timed call (milliseconds). */
typedef struct {
    double phase_ms;          /* densities + phase indicator kernel                         */
    double collide_ms;        /* fused gradient + collision + recolour + stream kernel       */
    double bc_ms;             /* pressure-face kernel (0 if unused)                          */
    double step_ms;           /* wall time per step between the first and last event         */
    int64_t phase_launches, collide_launches, bc_launches;
    double collide_parity_ms[2]; /* collide_ms over the even [0] and odd [1] AA steps alone    */
} lbm_timing;

/* Launch configuration of the two step kernels. block: threads per workgroup (64, 128 or 256);
 * schedule: 1 = workgroups take consecutive tiles of the pore list in launch order, 2 = XCD-aware
 * order: each of the 8 XCDs takes runs of consecutive tiles, the runs interleaved, so that
 * neighbouring tiles share an L2; 3 = the XCD-aware order run from the end of the pore list, so
 * that a kernel following one in forward order starts where that one ended (on lines that may
 * still be cached). run: the run length in tiles of schedules 2 and 3 (1 to 64; default 16), on
 * even [0] and odd [1] steps: the odd AA step's reads and writes land a neighbour away, so it
 * gains from longer runs (more of the lines it shares with nearby tiles stay on one XCD), the even
 * step from shorter ones. stream: 1 = the data a launch touches once (even-step populations, the
 * neighbour lookup, the moment slots, phi and N written for the next kernel) is read and written
 * with non-temporal hints, so the L2 keeps the lines neighbouring voxels re-read; right for
 * domains far larger than the 256 MB Infinity Cache, wrong for those it holds from one step to the
 * next. wg: at most this many workgroups of the kernel resident per CU (0: as many as its
 * registers allow; up to 16), enforced by reserving LDS the kernel does not use; fewer resident
 * waves keep more of the lines that neighbouring voxels share in the L2. When the domain's device
 * memory exceeds 512 MiB, lbm_domain_create sets stream = 1, the limits the autotuner picks at
 * 512^3 (phase / collide wg: FP64 5 / 2, FP32-mixed 5 / 3, FP32-dev 0 / 3) and collide runs of 4
 * (even) / 32 (odd) tiles; else stream 0, no limits and runs of 16. Results do not depend on the
 * configuration (bitwise). */
typedef struct {
    int32_t phase_block, phase_schedule;
    int32_t collide_block, collide_schedule;
    int32_t phase_stream, collide_stream;
    int32_t phase_wg, collide_wg;
    int32_t phase_run[2], collide_run[2];  /* [0]: even steps, [1]: odd steps                  */
    double phase_ms, collide_ms;  /* average per launch measured by lbm_autotune, else 0        */
} lbm_tuning;

typedef struct {
    int64_t n_pore;           /* pore voxels (the sparse list length N)                     */
    int64_t n_solid_tail;     /* solid voxels adjacent to a pore, plus the wall entry        */
    int64_t ld;               /* leading dimension of the SoA population arrays              */
    int64_t device_bytes;     /* device memory held by the domain                            */
    int64_t step;             /* completed steps                                             */
    int32_t precision;        /* lbm_precision                                               */
    int32_t block_size;       /* threads per workgroup in use                                */
    int32_t neighbour_mode;   /* LBM_NBR_TABLE, LBM_NBR_RANK or LBM_NBR_COMPACT              */
    int32_t compact_ex_waves; /* COMPACT: waves of 64 voxels kept as int32 entries; else 0    */
} lbm_domain_info;

/* Create a domain from a labelled image (sections "Initial conditions and wetting maps" and
 * "Modeling Wetting"): labels[nx*ny*nz] with values in [0, n_labels); label_kind[n_labels]
 * (lbm_label_kind); label_affinity[n_labels] (phi_s of solid labels, in [-1, 1]);
 * voxel_affinity (nullable, dense): per-voxel phi_s that overrides the label's for solid voxels;
 * init_phi (nullable, dense): initial phi in [-1, 1] of LBM_LABEL_PORE_INIT voxels (required if
 * any label has that kind). The initial state is rest equilibrium, rho = 1, u = 0,
 * N_a = (1 + phi)/2, N_b = (1 - phi)/2. alloc and hip_stream are nullable. On success *out owns
 * the domain. Errors: LBM_ERR_ARG (bad sizes, labels, parameters: tau <= 1/2, rho <= 0, no pore
 * voxel, beta outside (0,1), bc_z with a periodic z axis), LBM_ERR_OOM, LBM_ERR_DEVICE. */
lbm_status lbm_domain_create(const lbm_params* params, const int32_t* labels, int32_t n_labels,
                             const int8_t* label_kind, const double* label_affinity,
                             const double* voxel_affinity, const double* init_phi,
                             const lbm_allocator* alloc, void* hip_stream, lbm_domain** out);

/* Advance nsteps >= 0 time steps, asynchronously on the domain's stream (the time step of the
 * colour model: densities, phase indicator, colour gradient, MRT collision with the interfacial
 * terms and body force, recolouring, streaming with halfway bounce-back at solids). Records a
 * reduction every reduce_every steps. Returns LBM_ERR_UNSTABLE without stepping once a
 * reduction has seen a non-finite value. */
lbm_status lbm_step(lbm_domain* d, int64_t nsteps);

/* Same as lbm_step, but brackets every kernel launch with HIP events and reports the average
 * device time per launch of each kernel in *out. Synchronises. For measurement only. */
lbm_status lbm_step_timed(lbm_domain* d, int64_t nsteps, lbm_timing* out);

/* Copy one field (lbm_field) of the current state into host_dense[nx*ny*nz]; solid voxels are
 * set to NaN. Synchronises. */
lbm_status lbm_read_field(lbm_domain* d, int32_t field, double* host_dense);

/* Copy one field of the current state for the pore voxels only, in the library's pore order
 * (see lbm_pore_index), into host_pore[n_pore]. Synchronises. */
lbm_status lbm_read_pore_field(lbm_domain* d, int32_t field, double* host_pore);

/* Dense voxel index of each pore voxel, in the library's pore order: host_index[n_pore]. */
lbm_status lbm_pore_index(lbm_domain* d, int64_t* host_index);

/* Reduce the current state (see lbm_reduction). Synchronises. */
lbm_status lbm_reduce(lbm_domain* d, lbm_reduction* out);

/* Steady-state flow control (section "Steady-state" simulation protocol of the paper: total
 * capillary number, body-force adaptation F <- (Ca* / Ca) F capped at a factor of two, and the
 * steady-state test on the change of Ca over an interval t').
 *
 * lbm_set_force replaces the body force F (lattice units) from the next step on; for a pooled
 * domain, from its pool's next step. Errors: LBM_ERR_ARG for a null or non-finite force. */
lbm_status lbm_set_force(lbm_domain* d, const double force[3]);

typedef struct {
    double ca_target;     /* Ca* > 0: after relax_steps, F <- clamp(Ca* / Ca) F; 0 keeps F       */
    double max_factor;    /* bound of one rescaling: the factor lies in [1/max_factor,
                           * max_factor] (the paper uses 2); >= 1. Ca == 0 rescales by it    */
    double tol;           /* steady when |Ca(t) - Ca(t - interval)| / Ca(t) < tol               */
    int64_t relax_steps;  /* steps before the rescaling (also taken when ca_target == 0)       */
    int64_t interval;     /* t', steps between two Ca measurements of the steady test; > 0     */
    int64_t max_steps;    /* cap on the steps of this call (relaxation included); > 0          */
} lbm_steady_params;

typedef struct {
    int64_t steps;        /* steps taken by this call                                        */
    int32_t converged;    /* 1 if the steady test passed, 0 if max_steps was reached first   */
    int32_t rescales;     /* force rescalings applied (0 or 1)                               */
    double ca;            /* Ca of the final state                                           */
    double delta_ca;      /* last |Ca(t) - Ca(t - interval)| / Ca(t); -1 if never measured   */
    double factor;        /* the rescaling factor applied (1 if none)                        */
    double force[3];      /* body force at the end                                           */
    lbm_reduction last;   /* reduction of the final state                                    */
} lbm_steady_result;

/* Run one steady-state point: relax_steps steps, then (ca_target > 0) one force rescaling from
 * the measured Ca, then steps in blocks of `interval` with a Ca measurement after each, until
 * the relative change of Ca between two consecutive measurements falls below tol or max_steps
 * steps have been taken. Ca is the total capillary number of lbm_reduction (FP64). Synchronises
 * after each block. Errors: LBM_ERR_ARG (bad parameters), LBM_ERR_STATE (pooled domain: step
 * the pool), LBM_ERR_UNSTABLE (a measurement saw a non-finite value). */
lbm_status lbm_run_steady(lbm_domain* d, const lbm_steady_params* sp, lbm_steady_result* out);

/* Morphological growth of fluid a (section "Shell Aggregation Protocol"): the distance map
 * Phi_a of the fluid (negative inside a) is built from the phase field -- the closed form of
 * the equilibrium interface profile, -(1/(2 beta)) ln((1 + phi)/(1 - phi)), where
 * |phi| < tanh(band beta), elsewhere -/+(d - 1/2) with d the distance between voxel centres to
 * the nearest voxel across the boundary of {pore voxels with phi > 0} (solid voxels and the
 * outside of non-periodic faces lie outside it), searched within `radius`; the map is moved by
 * delta (> 0 dilates fluid a, < 0 erodes it), the phase becomes the equilibrium profile of the
 * moved map, phi' = 2 e / (1 + e) - 1 with e = exp(-2 beta (Phi_a - delta)) (voxels with
 * nothing across the boundary within the radius keep their phase), and the densities restart
 * at rest with N_a = N (1 + phi')/2, N_b = N (1 - phi')/2 and the voxel's current N. The flow
 * populations, the step counter and the history are kept. The first call allocates work
 * buffers (about 4.3 nx*ny*nz bytes plus 17 bytes per pore voxel) that stay with the domain.
 * Errors: LBM_ERR_ARG (parameters; also an image of 2^31 voxels or more, or an edge above
 * 16384), LBM_ERR_STATE (pooled domain), LBM_ERR_OOM. Synchronises. */
typedef struct {
    double delta;          /* growth distance in voxels; |delta| <= radius - 2; unused when
                            * target_ratio > 0                                               */
    double target_ratio;   /* > 0: delta for this ratio of the volume of fluid a, from a unit
                            * trial (delta = +-1) rescaled linearly, capped at radius - 2     */
    double band;           /* half-width of the closed-form band in voxels, in (0, radius]   */
    int32_t radius;        /* search radius of the far-field distance, 2..12                  */
    int32_t pad_;
} lbm_morph_params;

typedef struct {
    double delta;            /* growth distance applied                                      */
    int64_t volume_before;   /* pore voxels inside fluid a before (Phi_a < 0)                */
    int64_t volume_unit;     /* inside after the unit trial (target_ratio > 0), else 0       */
    int64_t volume_after;    /* inside the moved map (Phi_a - delta < 0)                      */
} lbm_morph_result;

lbm_status lbm_morph(lbm_domain* d, const lbm_morph_params* mp, lbm_morph_result* out);

/* Pore voxels with phi > 0 in the current state (the volume of fluid a). Synchronises. */
lbm_status lbm_phase_volume(lbm_domain* d, int64_t* volume);

/* The shell aggregation protocol: until the volume of fluid a has reached target_ratio times
 * its volume at the call (at least, when growing; at most, when shrinking), apply lbm_morph with
 * the remaining ratio as its target and relax for relax_steps LB steps; at most max_rounds
 * applications. */
enum { LBM_SHELL_MAX_DELTAS = 32 };
typedef struct {
    double target_ratio;   /* V_end / V_start of fluid a: > 1 grows it, < 1 shrinks it       */
    double band;           /* as in lbm_morph_params                                          */
    int32_t radius;        /* as in lbm_morph_params                                          */
    int32_t max_rounds;    /* >= 1                                                            */
    int64_t relax_steps;   /* LB steps after each application, >= 0                          */
} lbm_shell_params;

typedef struct {
    int32_t rounds;        /* applications made                                               */
    int32_t reached;       /* 1 if the target volume was reached                              */
    int64_t steps;         /* LB steps taken                                                  */
    int64_t volume_start, volume_end;   /* pore voxels with phi > 0 before and after          */
    double deltas[LBM_SHELL_MAX_DELTAS];  /* growth distance of each application (first 32)  */
} lbm_shell_result;

lbm_status lbm_shell_aggregate(lbm_domain* d, const lbm_shell_params* sp, lbm_shell_result* out);

/* Reductions recorded by lbm_step (every reduce_every steps) since the last call, oldest
 * first, at most max_count of them; *count receives the number written. Synchronises. */
lbm_status lbm_read_history(lbm_domain* d, lbm_reduction* out, int32_t max_count,
                            int32_t* count);

/* Serialise the state (populations, step counter) to host_buf. With host_buf == NULL only
 * *nbytes is set to the size needed. Errors: LBM_ERR_ARG if *nbytes is too small. */
lbm_status lbm_state_save(lbm_domain* d, void* host_buf, size_t* nbytes);

/* Restore a state written by lbm_state_save of a domain with the same geometry and precision.
 * Clears the sticky unstable flag. Errors: LBM_ERR_STATE on a size or header mismatch. */
lbm_status lbm_state_load(lbm_domain* d, const void* host_buf, size_t nbytes);

lbm_status lbm_domain_get_info(lbm_domain* d, lbm_domain_info* out);

/* Autotuner: times every (block, schedule, stream) candidate of each step kernel over
 * trial_steps >= 2 steps on this domain, then workgroup limits of 1 to 8 per CU on the best of
 * them, then (XCD-aware schedules) run lengths of 4 to 64 tiles for each step parity in turn,
 * applies the fastest, and writes it to *out (nullable).
 * The state, step counter and reduction history are restored afterwards, so the results of later
 * steps are unchanged. Synchronises; needs device memory for one copy of the populations
 * (LBM_ERR_OOM otherwise). */
lbm_status lbm_autotune(lbm_domain* d, int32_t trial_steps, lbm_tuning* out);

/* Apply a launch configuration (e.g. one cached from an earlier lbm_autotune on the same GPU,
 * precision and size class). LBM_ERR_ARG for an unsupported block, schedule, stream flag,
 * workgroup limit or run length. */
lbm_status lbm_set_tuning(lbm_domain* d, const lbm_tuning* t);
lbm_status lbm_get_tuning(lbm_domain* d, lbm_tuning* out);

/* Host-only: *bytes receives exactly the device memory lbm_domain_create would allocate for
 * these arguments (runs the CPU pre-pass; no GPU needed). For admission control by HBM budget
 * before anything is allocated. Same errors as lbm_domain_create's argument checks. */
lbm_status lbm_domain_footprint(const lbm_params* params, const int32_t* labels,
                                int32_t n_labels, const int8_t* label_kind,
                                const double* label_affinity, const double* voxel_affinity,
                                const double* init_phi, int64_t* bytes);

/* Host-only inspection of the sparse layout a domain would use (no GPU needed): runs the CPU
 * pre-pass on the same arguments as lbm_domain_create and reports *n_pore and *n_tail. Each
 * nullable output array, if given, must hold: pore_voxel[n_pore] (dense index of each pore
 * voxel, pore order), nbr[18 * n_pore] (row q-1 holds the neighbour of every pore voxel along
 * D3Q19 velocity q = 1..18: a pore index < n_pore, or n_pore + t for tail entry t, a solid or
 * wall neighbour), tail_phi[n_tail] (phi_s of each tail entry; entry 0 is the wall outside
 * non-periodic faces). Call once with NULL arrays to learn the sizes. The query also replays
 * the rank lookup (where it applies) and decodes the compact lookup for every pore voxel and
 * direction against this table, and returns LBM_ERR_STATE if they disagree (an internal error,
 * never expected). Only the image and its labels are checked here, not the fluid parameters. */
lbm_status lbm_prepass_query(const lbm_params* params, const int32_t* labels, int32_t n_labels,
                             const int8_t* label_kind, const double* label_affinity,
                             const double* voxel_affinity, const double* init_phi,
                             int64_t* n_pore, int64_t* n_tail, int64_t* pore_voxel,
                             int32_t* nbr, double* tail_phi);

/* Release all device memory of the domain and the handle itself. NULL is accepted. */
lbm_status lbm_domain_destroy(lbm_domain* d);

/* ---- Pools: many independent domains advanced together ----------------------------------
 * A pool steps every member domain with one launch per kernel per time step (a persistent grid
 * striding over the tiles of all members), in chunks captured once as a HIP graph and replayed.
 * Members keep their own state and parameters; a member's results are bitwise the same as
 * stepping it alone. A member with pressure faces (bc_z == 1) also gets its own boundary
 * launches (inlet density, face conditions) after the batched ones, so its admission or
 * retirement rebuilds the captured graph. Members must share the pool's precision and have the
 * same step parity as the pool (a fresh domain joins a pool whose step count is even). While a
 * domain is a member it runs on the pool's stream and lbm_step on it returns LBM_ERR_STATE; its
 * fields, reductions and state can still be read. The pool never frees member domains. */

/* Create a pool for up to max_slots members whose device memory (lbm_domain_info.device_bytes)
 * sums to at most hbm_budget_bytes. chunk_steps (even, >= 2) is the length of the captured step
 * chunk. alloc (nullable) is the device-memory hook for the pool's own tables (slot arguments,
 * tile and group tables, reduction partials: about 4 KiB + 25 KiB per slot), else hipMalloc;
 * members keep their own memory. hip_stream is nullable (the pool then owns a stream). */
lbm_status lbm_pool_create(int64_t hbm_budget_bytes, int32_t precision, int32_t max_slots,
                           int32_t chunk_steps, const lbm_allocator* alloc, void* hip_stream,
                           lbm_pool** out);

/* Add a domain; *slot receives its slot index. LBM_ERR_OOM if the budget or the slots are
 * exhausted; LBM_ERR_STATE for a precision or parity mismatch or a pooled domain. */
lbm_status lbm_pool_admit(lbm_pool* pool, lbm_domain* d, int32_t* slot);

/* Remove the member of `slot`: it keeps its state and returns to its own stream. *out
 * (nullable) receives its handle. The caller still owns the domain (the pool never frees one). */
lbm_status lbm_pool_retire(lbm_pool* pool, int32_t slot, lbm_domain** out);

/* Advance every member by nsteps >= 0 steps, asynchronously on the pool's stream. */
lbm_status lbm_pool_step(lbm_pool* pool, int64_t nsteps);

/* Reduce the member of `slot` now (see lbm_reduction), bitwise what lbm_reduce gives on it.
 * Synchronises. LBM_ERR_ARG for an empty slot. */
lbm_status lbm_pool_reduce(lbm_pool* pool, int32_t slot, lbm_reduction* out);

/* Reduce every member now (one batched launch). out[slot] is written for slots 0..max_count-1
 * (an empty slot gets n_pore = 0); *count receives the number of slots written. Synchronises.
 * Each member's values are bitwise those of lbm_reduce on it. */
lbm_status lbm_pool_reduce_all(lbm_pool* pool, lbm_reduction* out, int32_t max_count,
                               int32_t* count);

typedef struct {
    int32_t max_slots, members, chunk_steps, grid;  /* grid: workgroups of the batched launch */
    int64_t step, used_bytes, budget_bytes, tiles;
    int64_t graph_replays, eager_steps;
    int32_t order;            /* tile order of the batched launch (see lbm_pool_set_order)  */
    int32_t groups;           /* cache groups of the captured chunk (0: none; -1: not yet
                                 computed since the last membership change)                  */
} lbm_pool_info;
lbm_status lbm_pool_get_info(lbm_pool* pool, lbm_pool_info* out);

/* Cache groups: with group_bytes > 0 the captured chunk runs the members in groups, each a run
 * of consecutive members (slot order) whose lbm_domain_info.device_bytes sum to at most
 * group_bytes (a larger member forms a group of its own), and each group takes all chunk_steps
 * steps before the next group starts, so that a group sized to the last-level cache keeps its
 * state there across its steps. Eager steps (counts that are not whole chunks) still step all
 * members together. Members are independent, so results are bitwise the same for any
 * group_bytes; 0 (the default) turns grouping off. Takes effect at the next lbm_pool_step;
 * a change of the grouping rebuilds the captured graph. The pool keeps 4 * (max_slots + 1)
 * bytes of device memory per group for the group tables (LBM_ERR_OOM from lbm_pool_step if
 * they cannot be allocated). LBM_ERR_ARG for group_bytes < 0. */
lbm_status lbm_pool_set_group_bytes(lbm_pool* pool, int64_t group_bytes);

/* Set the number of workgroups of the batched step kernels (e.g. from an autotuner);
 * 0 restores the default (32 per compute unit). Invalidates the captured graph. */
lbm_status lbm_pool_set_grid(lbm_pool* pool, int32_t grid);

/* Tile order of the batched step kernels: 0 = tiles in launch order, 1 = XCD-aware order (each
 * of the 8 XCDs takes runs of 16 consecutive tiles, the runs interleaved; the launch is rounded
 * up to whole runs; the default). Results do not depend on it (bitwise). Invalidates the
 * captured graph. LBM_ERR_ARG for another value. */
lbm_status lbm_pool_set_order(lbm_pool* pool, int32_t order);

/* Autotuner for the batched launch: times each candidate workgroup count (multiples of the
 * compute-unit count) in both tile orders over trial_steps >= 2 steps of the current members
 * and applies the fastest pair; then, if the pool is at an even step, times one replay of the
 * captured chunk for each cache-group size (lbm_pool_set_group_bytes: 0, 128, 192, 256, 320 and
 * 384 MiB) and applies the fastest. Writes the workgroup count to *grid (nullable; the order
 * and the group count are in lbm_pool_info). Every member's state and step counter are
 * restored, so later results are unchanged. Needs device memory for one copy of the members'
 * populations. */
lbm_status lbm_pool_autotune(lbm_pool* pool, int32_t trial_steps, int32_t* grid);

/* Retire every member and free the pool. NULL is accepted. */
lbm_status lbm_pool_destroy(lbm_pool* pool);

/* ---- Image pre-processing (section "Initial conditions and wetting maps": morphological
 * drainage and the mixed-wet relabelling; section "Simulation protocol for steady-state flow":
 * the mixing region at the inlet and outlet). These turn a segmented image into the labels and
 * initial fluids of lbm_domain_create. Dense host images in and out (index x + nx*(y + ny*z));
 * the work runs on the current HIP device, on hip_stream (nullable: the null stream), with
 * device memory the call allocates and frees itself; every call is synchronous. Distances are
 * Euclidean between voxel centres, handled squared as exact integers. Sizes: 1 <= nx, ny, nz
 * <= 16384 and nx*ny*nz < 2^31. Errors: LBM_ERR_ARG (sizes, values), LBM_ERR_OOM,
 * LBM_ERR_DEVICE (no device, or a HIP call failed). */

/* Squared Euclidean distance transform: dist_sq[v] = min |v - w|^2 over the voxels w with
 * feature[w] != 0, counting periodic images on axes with periodic[a] != 0; bit a of wall_axes
 * (1: x, 2: y, 4: z) adds a plane of feature voxels just outside both faces of that axis when
 * it is not periodic. dist_sq[v] = -1 where there is no feature at all. */
lbm_status lbm_prep_distance(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                             int32_t wall_axes, const uint8_t* feature, int32_t* dist_sq,
                             void* hip_stream);

/* Allocation-free form of lbm_prep_distance, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * transform of the same arguments, but feature_dev[nx*ny*nz] and dist_sq_dev[nx*ny*nz] are
 * DEVICE pointers owned by the caller (dist_sq_dev 4-byte aligned), the call is asynchronous on
 * hip_stream (nullable: the null stream) and it allocates nothing: its work buffers live in a
 * fixed 16 MiB device array of the library, one per GPU, held until the process ends. The image
 * must fit that array: 8 bytes per 64-voxel row word (ny*nz*ceil(nx/64) words) plus 4 bytes per
 * voxel, e.g. up to about 3.9M voxels (a 157^3 image); LBM_ERR_ARG otherwise, before anything is
 * launched. Every call on one GPU uses the same array, so calls on that GPU must not overlap
 * (use one stream, or synchronise between calls). Errors as lbm_prep_distance, and
 * LBM_ERR_DEVICE if a launch fails. */
lbm_status lbm_prep_distance_noalloc(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                                     int32_t wall_axes, const uint8_t* feature_dev,
                                     int32_t* dist_sq_dev, void* hip_stream);

typedef struct {
    double target_sw;   /* water (wetting-fluid) saturation to reach, in [0, 1)              */
    int32_t inlet;      /* 1: only sphere centres connected through face-adjacent centres to */
                        /* the z = 0 plane count (needs periodic[2] == 0); 0: every centre   */
    int32_t pad_;
} lbm_drain_params;

typedef struct {
    int32_t radius_sq;      /* chosen k = R^2                                                */
    int32_t max_radius_sq;  /* largest D^2 over the pore voxels                              */
    int32_t evaluations;    /* drainage evaluations the radius search made                    */
    int32_t pad_;
    int64_t n_pore, n_nw;   /* pore voxels; voxels given to the non-wetting fluid             */
    double sw;              /* 1 - n_nw / n_pore                                             */
} lbm_drain_result;

/* Morphological drainage (the sphere-placing operation of Adalsteinsson and Hilpert, 2006,
 * which the paper uses for its initial fluid configurations). D(x) is the distance from pore
 * voxel x to the nearest solid voxel (pore[x] == 0), or to a plane of wall voxels just outside
 * each non-periodic face (except the two z faces when dp->inlet is set: those border the fluid
 * reservoirs). A sphere of radius R = sqrt(k) fits at x when D^2(x) >= k; the non-wetting
 * region is every pore voxel closer than R to a fitting centre (with dp->inlet, to a centre
 * connected to the z = 0 plane). k is the largest integer in [1, max D^2] whose water
 * saturation 1 - |nw| / |pore| is <= dp->target_sw, found by bisection over k; k = 1 when none
 * is. On success nw[nx*ny*nz] holds 1 on the non-wetting voxels and 0 elsewhere, and *out the
 * radius and counts. Extra errors: LBM_ERR_ARG with no pore voxel, or with neither a solid voxel
 * nor a wall (unbounded distances). */
lbm_status lbm_prep_drain(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                          const uint8_t* pore, const lbm_drain_params* dp, uint8_t* nw,
                          lbm_drain_result* out, void* hip_stream);

/* Mixed-wet relabelling: labels_out = labels, except that every solid voxel (label_kind of its
 * label == LBM_LABEL_SOLID) whose distance to the nearest voxel with nw != 0 (periodic images on
 * periodic axes) is at most dist takes new_label (the paper relabels within 2 voxel units of the
 * oil). labels in [0, n_labels); new_label >= 0 (it may be a label not yet in the table);
 * 0 <= dist <= 16384. labels_out may equal labels. */
lbm_status lbm_prep_relabel(int32_t nx, int32_t ny, int32_t nz, const int32_t periodic[3],
                            const int32_t* labels, int32_t n_labels, const int8_t* label_kind,
                            const uint8_t* nw, double dist, int32_t new_label,
                            int32_t* labels_out, void* hip_stream);

/* Mixing region along z: labels_out = labels, except that in the first nmix planes a solid
 * voxel takes pore_label where the last plane (z = nz-1) of labels is pore at the same (x, y),
 * and in the last nmix planes where the first plane (z = 0) is pore. 0 <= nmix <= nz;
 * pore_label in [0, n_labels) with a pore kind. labels_out may equal labels. */
lbm_status lbm_prep_mixing_layer(int32_t nx, int32_t ny, int32_t nz, const int32_t* labels,
                                 int32_t n_labels, const int8_t* label_kind, int32_t nmix,
                                 int32_t pore_label, int32_t* labels_out, void* hip_stream);

/* Message of the calling thread's last error ("" if none). Valid until its next call. */
const char* lbm_last_error(void);

/* Library version string. */
const char* lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
