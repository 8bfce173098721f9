/*
 * lbprint.h -- C ABI of the MI355X (gfx950) library for the regularized
 * colour-gradient lattice Boltzmann model of direct-writing printing
 * (Monteferrante, Montessori, Succi, Pisignano, Lauricella, arXiv:2102.02655).
 *
 * One simulation ("handle") advances two population sets -- ink (Y, the
 * paper's "yellow" colour) and air (B, "blue") -- on a D3Q19 lattice, or on
 * the paper's own D2Q9 lattice in the x-z plane (lb_params.lattice), with the
 * per-cell step of Sec. II.A-B:
 *   moments (Sec. II.A), the colour gradient (Eq. (lattgrad)) with wall
 *   densities (Eq. (wet)), the ink's local relaxation time from the strain
 *   rate (Eqs. (notnewvisc)-(tauofgammadot)) mixed by Eq. (tauinter), the
 *   regularised BGK collision (Eqs. (reg), (modbgk)) with exact-difference
 *   forcing, the perturbation (Eq. (pertopform)) and recolouring operators,
 *   streaming (Eq. (lbm)) with halfway bounce-back, moving-wall bounce-back
 *   (Eq. (movwall)), the nozzle inlet (Eq. (movnozzle)), anti-bounce-back
 *   pressure faces, and a moving print-head template whose released nodes are
 *   created at equilibrium and whose covered nodes are deleted.
 *
 * Conventions
 *   - Lattice units (dx = dt = 1).  Box nx * ny * nz; x and y are periodic;
 *     the z faces are periodic, walls or pressure faces.  Cell (x, y, z) has
 *     its centre at integer coordinates.
 *   - Field arrays are C order [z][y][x] (numpy shape (nz, ny, nx)); velocity
 *     arrays are [z][y][x][3].
 *   - Colour k = 0 is the ink Y, k = 1 the air B.
 *   - All calls return lb_status; nothing throws across the ABI.  A handle is
 *     not thread-safe; separate handles may share a stream.
 *
 * Memory ownership
 *   - The caller owns lb_params and every host array; they are read during
 *     the call and never retained.
 *   - The caller owns the device workspace: it allocates at least
 *     lb_footprint() bytes (256-byte aligned) and lends it exclusively to the
 *     handle until lb_destroy().  The library never allocates or frees device
 *     memory on this path.
 *   - The caller owns the HIP stream; every kernel and copy of a handle is
 *     enqueued on it.  lb_create(), lb_moments(), lb_timing_read() and
 *     lb_step() with check_interval > 0 synchronise it.
 */
#ifndef LBPRINT_H
#define LBPRINT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* inconsistent parameters, bad pointer or size           */
    LB_ENOMEM = -2,    /* workspace smaller than lb_footprint()                  */
    LB_EDEVICE = -3,   /* a HIP call failed (message in lb_last_error)           */
    LB_EUNSTABLE = -4, /* NaN, negative density or |u| > 0.3 detected            */
    LB_ESTATE = -5     /* call not allowed in the handle's state                 */
} lb_status;

/* Population storage.  LB_F64: FP64 storage and arithmetic.  LB_F32: FP32
 * storage and arithmetic (masses and conservation sums always in FP64).
 * LB_BF16_DEV and LB_F16_DEV (reduced storage, FP32 arithmetic): each
 * post-collision population is kept as its deviation from the equilibrium of
 * its source cell's post-collision moments (Sec. II.A, the modified
 * equilibrium), in BF16 or as FP16 of deviation / w_i, both colours of a link
 * packed in one 32-bit word, beside the cell's five moments (rho_Y, rho_B and
 * the forced velocity) in FP32.  Any other value: LB_EINVAL. */
typedef enum { LB_F64 = 0, LB_F32 = 1, LB_BF16_DEV = 2, LB_F16_DEV = 3 } lb_storage;

/* Ink rheology (Sec. II.B): constant tau_y; power law nu = K gdot^(n-1); Cross
 * law nu = nu_inf + (nu0 - nu_inf) / (1 + (lambda gdot)^m) (Eq. (notnewvisc),
 * the paper's flow index renamed m).  gdot is the paper's 2 |Gamma|. */
typedef enum { LB_NEWTONIAN = 0, LB_POWER_LAW = 1, LB_CROSS = 2 } lb_rheology;

typedef enum { LB_FACE_PERIODIC = 0, LB_FACE_WALL = 1, LB_FACE_PRESSURE = 2 } lb_face;

typedef struct {
    int nx, ny, nz;
    int storage;              /* lb_storage                                                */
    double alpha[2];          /* phi_0 of Y and B (Sec. II.A); 1/3 gives phi_i = w_i         */
    double rho0[2];           /* pure-phase densities rho_Y^0, rho_B^0 (phase field, lid)   */
    double A, beta;           /* perturbation amplitude (Eq. (pertopform)), recolouring beta */
    double eps_g;             /* regulariser of |grad rho^N| in the recolouring's cos(phi)  */
    double tau_b;             /* air relaxation time (> 1/2)                                */
    int rheology;             /* lb_rheology                                                */
    double tau_y;             /* Newtonian ink relaxation time                              */
    double K, n;              /* power law                                                  */
    double nu0, nu_inf, lambda, m; /* Cross law                                             */
    double tau_min, tau_max;  /* clamp of the ink relaxation time (tau_min > 1/2)           */
    double rho_eps;           /* floor of rho_Y in the strain-rate equation                 */
    double zeta_wall[2];      /* wetting affinity of the z walls, Eq. (wet)                 */
    double zeta_noz[2];       /* wetting affinity of the nozzle                             */
    double drag_gamma;        /* substrate drag -gamma rho_Y (u - u_wall), Sec. II.B        */
    double drag_range;        /* drag acts where z + 1/2 < drag_range above a z-low wall    */
    double body_g[3];         /* body acceleration                                          */
    int face_zlo, face_zhi;   /* lb_face; both periodic or both not                         */
    double u_zlo[3], u_zhi[3];     /* wall velocities                                       */
    double rho_zlo[2], rho_zhi[2]; /* densities imposed by pressure faces (Y, B)            */
    int has_nozzle;           /* print head present (requires a non-periodic top face)      */
    double noz_x0[2];         /* head axis (x, y) at step 0                                 */
    double noz_v[2];          /* head velocity (x, y), constant (Sec. II.B)                 */
    double noz_r_in;          /* bore radius                                                */
    double noz_wall;          /* shell thickness                                            */
    double noz_tip_z;         /* shell from z >= noz_tip_z through the top face             */
    double u_ink[3];          /* ink velocity in the head frame, Eq. (movnozzle)            */
    double lid_rho_y;         /* ink density imposed on the inlet lid                       */
    int check_interval;       /* 0: checks only in lb_moments; k > 0: every k steps          */
    int lattice;              /* 0 or 19: D3Q19.  9: D2Q9 (Sec. II.A) in the x-z plane of a
                               * box with ny == 1; storage LB_F64 or LB_F32; every y
                               * component (body_g, u_zlo, u_zhi, u_ink, noz_v, noz_x0)
                               * must be 0; not a member of an lb_batch                      */
} lb_params;

typedef struct {
    double mass[2];           /* sum of rho_Y, rho_B over fluid cells, now (FP64)            */
    double mom[3];            /* sum of rho u (bare, without the half-force) over fluid cells */
    double mass_wall[2];      /* cumulative mass added by bounce-back / lid links            */
    double mass_open[2];      /* cumulative mass added by anti-bounce-back links             */
    double mass_created[2];   /* cumulative mass of nodes created by the moving head         */
    double mass_deleted[2];   /* cumulative mass of nodes deleted by the moving head         */
} lb_conserved;
/* mass[k](t) - mass[k](0) = mass_wall + mass_open + mass_created - mass_deleted,
 * to rounding. */

typedef struct lb_handle lb_handle;

/* Bytes of device workspace a handle needs for these parameters (pure host
 * computation; used for admission).  Includes the padding between population
 * planes (256 B, or 1 MiB + 256 B for planes of 16 MiB and more) and the
 * boundary-only arrays (moment sets, colour fields and macro fields of the
 * cells next to the z faces and the head), which a D3Q19 box with z walls
 * keeps for three layers at each face and a window of columns around the
 * head (the smallest power of two dividing nx, resp. ny, of at least
 * 2 ceil(r_out) + 16, else the whole extent; head speed at most 1/2 per
 * step), and
 * a periodic box, a faster head or a D2Q9 box for every cell.  LB_EINVAL on
 * bad parameters. */
lb_status lb_footprint(const lb_params *p, size_t *bytes);

/* Create a simulation.  rho_y, rho_b: host FP64 [z][y][x] initial densities;
 * u: host FP64 [z][y][x][3] initial velocity or NULL for rest.  The state is
 * f^k = f^{k,eq}(rho^k, u) at the fluid cells of step 0 (Sec. II.A).
 * dev_workspace: device pointer to ws_bytes >= lb_footprint() bytes.
 * hip_stream: the hipStream_t to enqueue on (NULL = default stream).
 * On success *out is a new handle; on failure *out is NULL. */
lb_status lb_create(const lb_params *p, const double *rho_y, const double *rho_b, const double *u,
                    void *dev_workspace, size_t ws_bytes, void *hip_stream, lb_handle **out);

/* Advance nsteps time steps (Eq. (lbm)); asynchronous on the handle's stream.
 * LB_ESTATE after an LB_EUNSTABLE result. */
lb_status lb_step(lb_handle *h, int nsteps);

/* Batched stepping: advance handle hs[i] by nsteps[i] steps, i = 0 .. n-1
 * (distinct handles; any mix of sizes, storage forms and parameters;
 * check_interval must be 0).  A handle's first step and an odd remainder run
 * as ordinary launches; the even part is ONE launch of a HIP graph holding
 * that many steps of the handle (captured once on a private stream,
 * instantiated, and cached in the handle -- at most four chains, keyed by
 * the step count and the step parity -- then replayed on every later call
 * with the same count).  Everything is enqueued on each handle's own stream,
 * so handles on different streams run concurrently.  The result of every
 * handle is bit-identical to stepping it alone with lb_step.  Asynchronous;
 * LB_EINVAL on bad arguments, LB_ESTATE on an unstable handle, LB_EDEVICE if
 * a graph call fails.  The cached graphs are released by lb_destroy. */
lb_status lb_step_batch(lb_handle *const *hs, const int *nsteps, int n);

/* Batches (serving, a parameter sweep of many simulations): one launch of
 * each step kernel advances every member of a batch.  A batch holds a slot
 * table in device memory -- per member its parameters, its buffers for both
 * step parities and the range of blocks it owns in each kernel's grid -- and
 * one HIP graph of k steps of the five batched kernels (boundary preparation,
 * node creation, wall densities, ghost layers, the fused step), captured once
 * and replayed; it is captured again only when the step count or a kernel's
 * block count outgrows it.  Every block runs its member's kernel body with
 * its block index within the member's share, which is the grid the member
 * uses alone, so every member's fields and FP64 sums are bit-identical to
 * stepping it alone with lb_step.
 *
 * lb_batch_footprint: bytes of device workspace a batch needs (the slot table
 * of at most 64 members; pure host computation).
 * lb_batch_create: storage is the lb_storage form every member must have;
 * dev_workspace (>= lb_batch_footprint bytes, 256-byte aligned) is lent to the
 * batch until lb_batch_destroy; hip_stream is the batch's stream.  The batch
 * also keeps two pinned host buffers for staging the table (hipHostMalloc).
 * lb_batch_step: advance hs[i] by nsteps[i] steps (n <= 64 distinct handles of
 * the batch's storage form, any sizes and parameters, check_interval 0).  A
 * member's first step (it reads its initial state) runs as an ordinary launch;
 * the rest run in the graph, where a member with fewer steps than the graph
 * sits out the later ones.  The batch stream waits for each member's stream
 * first, and each member's stream waits for the batch afterwards, so calls
 * on the handles keep their order.  Asynchronous; LB_EINVAL on bad arguments,
 * LB_ESTATE for an unstable member, LB_EDEVICE if a HIP call fails (message in
 * lb_batch_last_error).  The table is rebuilt at every call, so members may
 * join, leave or be destroyed between calls.
 * lb_batch_destroy: waits for the batch stream, releases the graph, events and
 * staging buffers (not the workspace or the members). */
typedef struct lb_batch lb_batch;
lb_status lb_batch_footprint(size_t *bytes);
lb_status lb_batch_create(int storage, void *dev_workspace, size_t ws_bytes, void *hip_stream, lb_batch **out);
lb_status lb_batch_step(lb_batch *b, lb_handle *const *hs, const int *nsteps, int n);
lb_status lb_batch_destroy(lb_batch *b);
const char *lb_batch_last_error(const lb_batch *b);

/* Fields and conserved sums at the current step.  rho_y, rho_b (N values) and
 * u (3N values, the physical velocity (sum f c + F/2) / rho) are written as
 * FP64 (dtype 0) or FP32 (dtype 1) into host (dst_is_device = 0) or device
 * (dst_is_device = 1) memory; any may be NULL.  Solid cells read 0.  cons may
 * be NULL.  Synchronises the stream.  Returns LB_EUNSTABLE (after filling the
 * outputs) if a NaN, a negative density or |u| > 0.3 is present. */
lb_status lb_moments(lb_handle *h, void *rho_y, void *rho_b, void *u, int dst_is_device, int dtype,
                     lb_conserved *cons);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): lb_moments
 * with the same arguments, outputs and errors, whose per-call partial sums
 * (pending boundary fluxes, deletions and creations, the fields' block sums,
 * the final values) live in a file-scope device array of the library instead
 * of the handle's workspace.  The array is 102.5 KB (12,816 doubles) and does
 * not grow with the box: the read-out kernels run a fixed grid of at most
 * 1,024 blocks, so no box is too large for it (LB_EINVAL guards the slot
 * counts).  Each GPU holds its own copy until the process ends; its address
 * on a device is taken once, when the first handle on that device is created
 * (LB_EDEVICE from this call if that failed).  The call allocates and frees
 * nothing.  Every call on one GPU shares the array: calls that overlap on one
 * GPU (different streams or threads) race and must be serialised by the
 * caller.  Host outputs are staged in the handle's spare population buffer,
 * as in lb_moments. */
lb_status lb_moments_noalloc(lb_handle *h, void *rho_y, void *rho_b, void *u, int dst_is_device, int dtype,
                             lb_conserved *cons);

/* Printing observables of Sec. IV on the x-z section y = w->y (0 on D2Q9),
 * at the current step.  A cell is ink where rho^N > 0, i.e. rho_Y rho_B^0 >
 * rho_B rho_Y^0 (FP64 masses); cells of the head are excluded.  The printed
 * thread is the ink in the window of columns x_lo .. x_lo + x_len - 1
 * (periodic) below z_hi (usually the nozzle tip plane, so that ink still in
 * the nozzle does not count); the window behind the moving nozzle is the
 * caller's choice.  Outputs (lattice units):
 *   ink_area   A_i: thread cells;
 *   height     h: 1 + the highest thread cell's z (the substrate wall lies
 *              at z = -1/2, so this is the thread's top above it);
 *   width      1 + the span of thread columns within the window;
 *   coverage   A_i / A_r with A_r = h * width, the circumscribing rectangle
 *              (0 if there is no thread);
 *   dp_max     the largest p - p0 over the section's ink cells, p = sum_k
 *              rho_k c_{s,k}^2 (Eq. (cgoef)'s partial pressures; 0 without
 *              ink);
 *   p0         rho_B^0 c_{s,B}^2, the pressure of air at rest;
 *   substrate_ink  ink cells in the layer z = 0 (first contact when > 0).
 * The POI of Sec. IV, (A_i / A_r) d / (h dp_max), and its normalisation over a
 * sweep are formed by the caller.  Runs the read-out's pull (as lb_moments;
 * the handle's read-out slots in its workspace) and synchronises the stream.
 * LB_EINVAL for a bad window (x_len < 1 or > nx, y outside the box). */
typedef struct {
    int x_lo, x_len;
    int z_hi;
    int y;
} lb_window;

typedef struct {
    double ink_area, height, width, coverage;
    double dp_max, p0;
    double substrate_ink;
} lb_observables;

lb_status lb_observe(lb_handle *h, const lb_window *w, lb_observables *out);

/* Current step count. */
long lb_time(const lb_handle *h);

/* Measurement aid: kernel timing with HIP events on the handle's stream.
 * lb_timing(h, 1) starts recording, at every following step, an event before
 * the step's first kernel, one before the fused step kernel and one after it;
 * lb_timing(h, 0) stops recording (what was recorded stays readable).
 * lb_timing_read() waits for the recorded events, returns the summed duration
 * of the fused step kernel (step_ms), of the boundary preparation kernels
 * that precede it (prep_ms) and the number of timed steps, then clears the
 * record.  Any output pointer may be NULL.  LB_EDEVICE if a HIP event call
 * fails (the events are host-side runtime objects; no device memory). */
lb_status lb_timing(lb_handle *h, int enable);
lb_status lb_timing_read(lb_handle *h, double *step_ms, double *prep_ms, long *steps);

/* Release the handle (host memory and its cached graphs; waits for the
 * handle's stream if graphs were cached; the workspace stays the caller's). */
lb_status lb_destroy(lb_handle *h);

const char *lb_strerror(lb_status s);
/* Last error message of a handle, or of the calling thread when h is NULL. */
const char *lb_last_error(const lb_handle *h);

#ifdef __cplusplus
}
#endif
#endif
