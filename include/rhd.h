/*
 * rhd.h -- C interface of the MI355X (gfx950) library for the gray two-moment (M1)
 * radiation-hydrodynamics method of Skinner & Ostriker (2013), "A two-moment
 * radiation hydrodynamics module in Athena using a time-explicit Godunov method".
 *
 * One call of rhd_step advances one operator-split gas step of the method (Sec. 3.1,
 * algorithm steps 2-6):
 *   1. implicit gas-radiation energy exchange over dt_gas (Sec. 3.4,
 *      Eqs. source:energyexchange to source:polynomial), per cell, in FP64;
 *   2. gas Van Leer step with the explicit gas sources (Eq. algorithm:gastransport,
 *      Eq. algorithm:source:explicit:gas);
 *   3. nsub radiation Van Leer subcycles of dt_gas/nsub with the gas frozen
 *      (Eq. algorithm:radtransport): M1 closure (Eqs. m1:m1tns, m1:chi), HLL fluxes
 *      (Eq. hyperbolic:hllflux2) bounded by the M1 eigenvalues
 *      (Eq. hyperbolic:evals13), unsplit conservative update, theta-scheme flux
 *      absorption (Eq. source:stiff:radmomentum:soln) and explicit sources;
 *   4. second-order correction of the gas sources with the radiation at t^{n+1}
 *      (Sec. 3.4, last displayed equation);
 *   5. an FP64 ledger of E + (c/chat) E_r, m + F/(c chat) and rho (Sec. 2.1) and a
 *      non-finite check of the state.
 *
 * Conventions for every function:
 *  - Status codes: RHD_OK (0) or a negative RHD_E* value; rhd_last_error() then
 *    holds a message. A failed call leaves the state as it was unless stated.
 *  - Host arrays belong to the caller; the library copies them in and out in FP64,
 *    structure-of-arrays, cell (i, j, k) at flat index i + nx*(j + ny*k). Vector
 *    fields (momentum, flux) are three consecutive blocks of nx*ny*nz values (x, y,
 *    z components). Device memory belongs to the handle.
 *  - Work is enqueued on the handle's HIP stream and returns before the GPU is done
 *    unless the function says it synchronises.
 *  - A handle is not thread-safe: use one handle per host thread and stream.
 */
#ifndef RHD_H
#define RHD_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RHD_OK            0
#define RHD_EINVAL       -1   /* bad argument: sizes, dt <= 0, nsub < 0, chat <= 0, theta */
#define RHD_ECFL         -2   /* chat * dt_gas / nsub > K0 * min(dx, dy, dz)               */
#define RHD_ENONFINITE   -3   /* a non-finite value appeared in the state                   */
#define RHD_ENOMEM       -4   /* device allocation failed                                   */
#define RHD_EDEVICE      -5   /* a HIP call failed; rhd_last_error() has the HIP message    */
#define RHD_ESTATE       -6   /* call out of order (e.g. rhd_step before rhd_set_state)     */
#define RHD_ETIMEOUT     -7   /* rhd_server_wait: the request did not finish in time         */

/* boundary kinds for rhd_params.bc[6] = {x-, x+, y-, y+, z-, z+} */
#define RHD_BC_PERIODIC   0
#define RHD_BC_OUTFLOW    1   /* zero-gradient copy of the edge cell                        */
#define RHD_BC_REFLECT    2   /* mirror image; the normal momentum and flux change sign     */
#define RHD_BC_FIXED      3   /* fixed radiation state (rhd_set_boundary) in every ghost cell
                                 beyond the face, in U^m and U^{m+1/2}; a cell beyond several
                                 fixed faces takes the last in the order x, y, z. The gas
                                 continues zero-gradient. Needs RHD_RAD_ONLY; such handles
                                 run the face-split or per-cell radiation kernels (not the
                                 tiled ones) and cannot join a batch.
                                 For driven problems such as the Marshak wave (Sec. 4.1.3). */

/* rhd_params.flags */
#define RHD_ISOTHERMAL          (1u << 0)  /* P = rho iso_cs^2, no gas energy equation     */
#define RHD_EXCHANGE_MASK       (3u << 1)
#define RHD_EXCHANGE_FULL       (0u << 1)  /* implicit exchange on dt_gas (Sec. 3.4)       */
#define RHD_EXCHANGE_ABSORB_ONLY (1u << 1) /* absorption only, on each radiation stage,
                                              Eq. source:stiff:radenergy:soln              */
#define RHD_EXCHANGE_NONE       (2u << 1)  /* radiative equilibrium: no exchange (Sec. 3.4) */
#define RHD_BETA_TAU            (1u << 3)  /* keep the O(beta tau) velocity terms
                                              (Eq. m1:simplifiedsource and S_e)            */
#define RHD_RAD_ONLY            (1u << 4)  /* gas frozen: no gas transport, no correction  */
#define RHD_PRECISION_MIXED     (1u << 5)  /* FP32 storage and stencils, FP64 exchange and
                                              ledger; without it everything is FP64. The
                                              face fluxes form chat^2 c E_r in FP32: state
                                              the problem in units where that stays well
                                              below 3e38 (cgs values of dense, hot gas can
                                              overflow it)                                 */
#define RHD_OPACITY_LAW         (1u << 7)  /* kappa_P = kappa_F = k0 (T_gas/T0)^a (rho/rho0)^b
                                              (Sec. 4.1.1), kappa_law = {k0, T0, rho0, a, b},
                                              from the gas state at the start of each gas
                                              step (and for rhd_suggest_dt); the kappa
                                              arrays of rhd_set_state are then not read   */
#define RHD_GAS_CV_T3           (1u << 6)  /* heat capacity c_v = cv_alpha T^3 (Sec. 4.1.3):
                                              a_R T^4 = (4 a_R / cv_alpha) e, so the exchange
                                              (theta-scheme of Eq. source:energyupdate) is
                                              linear in e. Needs RHD_RAD_ONLY, ideal gas   */
#define RHD_CLOSURE_P1          (1u << 8)  /* Eddington (P1) closure instead of M1: T = I/3
                                              and the fixed wave speeds +-chat/sqrt(3) in
                                              every face flux (Sec. 2.3; the comparison run
                                              of Sec. 4.3.5). The flux clamp |F| <= c E_r
                                              after each stage still applies              */

typedef struct {
  int nx, ny, nz;               /* interior cells; a dimension with n = 1 is inactive      */
  double dx, dy, dz;            /* uniform cell widths                                      */
  double gamma;                 /* ratio of specific heats (ignored when isothermal)        */
  double c_light;               /* c: ratio of photon energy to momentum, used in sources   */
  double a_rad;                 /* radiation constant a_R                                   */
  double r_gas;                 /* k_B / mu, so that P = rho r_gas T (Eq. momenteqns:perfectgas) */
  double iso_cs;                /* isothermal sound speed (RHD_ISOTHERMAL only)             */
  double cfl;                   /* Courant number K0 (Eq. algorithm:gastimestep), 0 < K0 <= 1 */
  double theta_E;               /* theta of the exchange update, in [0.5, 1] (Eq. source:energyupdate) */
  double theta_F;               /* theta of the flux absorption, in [0.5, 1]
                                   (Eq. source:stiff:radmomentum:soln)                      */
  double newton_rtol;           /* relative tolerance epsilon of the root solve, (0, 1)     */
  int newton_maxit;             /* Newton iterations before bisection takes over, >= 0      */
  double rho_floor, p_floor, er_floor;  /* floors for rho, P and E_r, >= 0                  */
  int bc[6];                    /* RHD_BC_* per face x-, x+, y-, y+, z-, z+; periodic faces
                                   come in pairs; reflecting faces need n >= 3             */
  unsigned flags;               /* RHD_* flags above                                        */
  double cv_alpha;              /* alpha of c_v = alpha T^3 with RHD_GAS_CV_T3, else unused */
  double kappa_law[5];          /* k0 >= 0, T0 > 0, rho0 > 0, a, b of RHD_OPACITY_LAW      */
} rhd_params;

typedef struct {
  double ledger[5];             /* after the last step or rhd_ledger: sum(E + (c/chat) E_r) dV,
                                   sum(m_x,y,z + F_x,y,z / (c chat)) dV, sum(rho) dV (FP64)  */
  double vmax;                  /* v_max of the last rhd_suggest_dt                         */
  long long exch_theta1;        /* cells whose exchange was redone with theta = 1           */
  long long exch_bisect;        /* cells whose exchange root needed bisection               */
  long long newton_iters;       /* total Newton iterations                                  */
  long long newton_max;         /* largest iteration count in one cell                      */
  long long rad_fclamp;         /* interior cells whose |F| was scaled back to c E_r        */
  long long rad_efloor;         /* interior cells raised to er_floor                        */
  long long gas_rhofloor;       /* interior cells raised to rho_floor                       */
  long long gas_pfloor;         /* interior cells raised to p_floor                         */
  long long nonfinite;          /* non-finite values seen by the last ledger pass           */
  long long first_nonfinite_cell; /* lowest flat cell index holding one, or -1              */
  long long steps;              /* gas steps taken                                          */
  long long subcycles;          /* radiation subcycles taken                                */
} rhd_diag;

/* Per-kernel GPU time measured with HIP events on the handle's stream (rhd_set_timing). */
#define RHD_TIMING_MAX 12
typedef struct {
  int nkernels;                          /* entries used                                   */
  char name[RHD_TIMING_MAX][24];         /* kernel names: exchange, gas_predict, ...       */
  long long calls[RHD_TIMING_MAX];       /* launches timed                                 */
  double total_ms[RHD_TIMING_MAX];       /* summed event-to-event duration                 */
  long long cells[RHD_TIMING_MAX];       /* cells processed per launch (padded regions for
                                            the predictors)                               */
} rhd_timing;

typedef struct rhd rhd_t;

/* Default parameters for an nx x ny x nz grid: unit box, gamma = 5/3, c = a_R = r_gas = 1,
   K0 = 0.4, theta_E = 1, theta_F = 0.51, epsilon = 1e-10, 50 Newton iterations, periodic
   faces, full exchange, FP64. Never fails. */
void rhd_default_params(rhd_params* p, int nx, int ny, int nz);

/* Create a handle: validates p (RHD_EINVAL), selects the current HIP device and
   allocates every device buffer the steps need (RHD_ENOMEM), so that rhd_step never
   allocates. hip_stream is a hipStream_t to enqueue on, or NULL for a stream the
   handle creates and owns. On failure *out is NULL. */
int rhd_create(const rhd_params* p, void* hip_stream, rhd_t** out);

/* Copy a state in (host FP64 arrays, layout above): rho (N), mom (3N), E (N, gas total
   energy; ignored when isothermal), Er (N), Fr (3N). kappaP and kappaF are the
   Planck-mean and flux-mean specific opacities: N values each, or one value each when
   kappa_scalar is 1. kappa_P multiplies the exchange term (a_R T^4 - E_r) and kappa_F
   every F and v term (Sec. 2.1, Eq. mixedframe:kappas). In mixed precision the values
   are rounded to FP32 (to nearest) on the host. Host arrays travel through pinned host
   chunks the library shares among all handles (two of 4 MiB per transfer in progress,
   kept until the process ends). Synchronises. */
int rhd_set_state(rhd_t* h, const double* rho, const double* mom, const double* E,
                  const double* Er, const double* Fr, const double* kappaP,
                  const double* kappaF, int kappa_scalar);

/* Same as rhd_set_state with every pointer in device memory of the handle's device
   (e.g. a torch tensor's data pointer). Enqueued on the stream, no synchronisation;
   the caller keeps the arrays alive until the stream has passed this call. */
int rhd_set_state_device(rhd_t* h, const double* rho, const double* mom, const double* E,
                         const double* Er, const double* Fr, const double* kappaP,
                         const double* kappaF, int kappa_scalar);

/* Emissivity j per cell (N host values), or NULL to remove it. It adds (chat/c) j to
   dE_r/dt, so that div F = j in a steady state (Sec. 4.3.6, Eq. radshell:sourceprofile).
   Synchronises. */
int rhd_set_emission(rhd_t* h, const double* j);

/* Radiation state U = (E_r, F_x, F_y, F_z) that the RHD_BC_FIXED face `face` (0..5 =
   x-, x+, y-, y+, z-, z+) holds from the next rhd_step on; it stays until set again
   (zero until the first call). A driven boundary sets it before each step, e.g. from
   Eq. marshak:suolson and the Marshak condition c E_r + 2 F = 4 F_inc of Sec. 4.1.3.
   RHD_EINVAL if the face is not a fixed face of an active dimension, or E_r <= 0, or a
   value is not finite. Host-side only. */
int rhd_set_boundary(rhd_t* h, int face, const double U[4]);

/* Advance one gas step of dt_gas with nsub radiation subcycles of dt_gas/nsub each
   (Sec. 3.1 steps 2-6, Eq. algorithm:radtimestep). chat is the reduced speed of light
   of this step (Sec. 3.2). nsub = 0 advances the exchange and the gas only.
   RHD_EINVAL for dt_gas <= 0, chat <= 0 or nsub outside [0, 2^20]; RHD_ECFL when
   chat * dt_gas / nsub > K0 * min(dx, dy, dz) (relative slack 1e-12); RHD_ESTATE
   before rhd_set_state. Asynchronous: errors found on the GPU (non-finite values)
   are reported by rhd_sync and rhd_get_diagnostics. */
int rhd_step(rhd_t* h, double dt_gas, double chat, int nsub);

/* Advance nsteps gas steps in one call: step k takes dt_gas[k] with nsub[k] radiation
   subcycles at the reduced speed of light chat, and, when bvals is not NULL, each
   RHD_BC_FIXED face holds bvals[24 k + 4 f .. 24 k + 4 f + 3] = (E_r, F_x, F_y, F_z) of
   face f during step k (entries of other faces are ignored; with bvals NULL the states
   of rhd_set_boundary stay). The result equals nsteps calls of rhd_set_boundary and
   rhd_step, bit for bit, with the ledger taken once at the end; afterwards the fixed
   faces keep the last step's states. A 1D RHD_RAD_ONLY grid of at most 1024 cells (2048
   in mixed precision) runs 1024 steps per launch of one workgroup (at such sizes
   separate launches cost more than the arithmetic); on its first such call the handle
   allocates its step tables (device and pinned host memory, 2 x 1024 steps). Other
   grids enqueue the steps one by one.
   Every step is checked before anything is enqueued: RHD_EINVAL for nsteps < 0, NULL
   arrays, dt_gas <= 0, nsub < 0, chat <= 0 or a fixed-face state with E_r <= 0 or a
   non-finite value; RHD_ECFL as rhd_step. Asynchronous like rhd_step. */
int rhd_run(rhd_t* h, int nsteps, const double* dt_gas, const int* nsub, double chat,
            const double* bvals);

/* Radiation-modified CFL step of the current state (Eqs. algorithm:ceff and
   algorithm:gastimestep): v_max = max(|v| + c_eff), dt_gas = K0 min(dx) / v_max,
   nsub = ceil(chat / v_max) (at least 1). Synchronises. */
int rhd_suggest_dt(rhd_t* h, double chat, double* dt_gas, int* nsub);

/* Recompute the FP64 ledger of the current state with the given chat (the step does
   this itself with its own chat). Asynchronous; read it with rhd_get_diagnostics. */
int rhd_ledger(rhd_t* h, double chat);

/* Copy the state out into host FP64 arrays laid out as for rhd_set_state (through the
   same pinned chunks). Any pointer may be NULL to skip that field. Synchronises. */
int rhd_get_state(rhd_t* h, double* rho, double* mom, double* E, double* Er, double* Fr);

/* Same as rhd_get_state into device FP64 arrays. Enqueued, no synchronisation. */
int rhd_get_state_device(rhd_t* h, double* rho, double* mom, double* E, double* Er,
                         double* Fr);

/* Counters accumulated since rhd_create or rhd_reset_diagnostics, the last ledger and
   v_max. Synchronises. */
int rhd_get_diagnostics(rhd_t* h, rhd_diag* out);

/* Zero the counters. Asynchronous. */
int rhd_reset_diagnostics(rhd_t* h);

/* Wait for the handle's stream. Returns RHD_ENONFINITE if the last ledger pass found
   a non-finite value, RHD_EDEVICE on a HIP error. */
int rhd_sync(rhd_t* h);

/* Start (enable = 1) or stop (0) timing every kernel launch of the handle with a pair of
   HIP events recorded on its stream; starting also clears the totals. Events come from a
   pool created on first use; a full pool is drained with one stream synchronisation. */
int rhd_set_timing(rhd_t* h, int enable);

/* Totals since timing was started. Synchronises. */
int rhd_get_timing(rhd_t* h, rhd_timing* out);

/* Kernel variants of the radiation subcycle (rhd_set_kernel_variant). */
#define RHD_KERNELS_PER_CELL  0   /* one thread per cell, every face flux evaluated twice     */
#define RHD_KERNELS_TILED     1   /* x-y tiles in LDS marching along z, every face flux once;
                                     3D grids without fixed faces only: other 2D and 3D
                                     grids run the face-split kernels up to 2^17 cells, the
                                     per-cell ones beyond; 1D grids along x of up to 512
                                     cells (FP64) or 1024 (mixed) run all subcycles of a step
                                     in one workgroup when the step has several or the grid
                                     at most 256 cells, other 1D steps the per-cell kernels */
#define RHD_KERNELS_FACE_SPLIT 2  /* 64 cells per block, one wavefront per face of a cell,
                                     fluxes met in LDS: for small grids of any dimension    */

/* Select the kernels of the radiation subcycle: variant RHD_KERNELS_*, tile_rows the
   rows of a 64-wide tile (4, 8 or 16; FP64 handles 4 or 8), zchunk the z-planes one tile
   walks (>= 1). In mixed precision the predictor stage always runs 4-row tiles of at most
   11 planes (its fastest shape on every grid measured) and tile_rows and zchunk set the
   corrector's and the gas stages'. Defaults after rhd_create: tiled, 8 rows, 8 planes. Results do not
   depend on the choice beyond rounding. RHD_EINVAL for values outside these sets. The
   tiled kernels address with 32-bit byte offsets: a grid whose padded arrays
   ((nx + 4)(ny + 4)(nz + 4) cells) exceed 4 GiB each (beyond ~1000^3 cells in mixed
   precision, ~800^3 in FP64) runs the per-cell kernels, and asking for the tiled ones
   there is RHD_EINVAL. The face-split kernels index cells with 32-bit integers (any grid
   rhd_create accepts). */
int rhd_set_kernel_variant(rhd_t* h, int variant, int tile_rows, int zchunk);

/* HIP graphs for the radiation subcycles (enable = 1; 0, the default, launches each
   kernel). With graphs on, the nsub-subcycle loop of rhd_step and rhd_run is captured
   from the handle's stream into a HIP graph the first time a key (nsub, dt_gas/nsub,
   chat, kernel choice) is seen and replayed while the key holds: steps of a fixed size
   cost one graph launch instead of 2 nsub kernel launches. A new key is captured again
   and written into the same executable graph. Results are the same bit for bit as
   without graphs (same kernels, same arguments). Not while kernel timing is on (the
   loop then launches directly). RHD_EINVAL for a handle on the null stream. */
int rhd_set_graph(rhd_t* h, int enable);

/* Subcycle-loop graphs captured and replayed by this handle so far. */
int rhd_get_graph_stats(const rhd_t* h, long long* captures, long long* replays);

/* Pick the fastest radiation-subcycle kernels for this handle's grid by timing them:
   every variant and tile shape (tile rows x z chunk) runs `reps` subcycles of dt_rad on
   the current state with HIP events, and the fastest becomes the handle's choice (see
   rhd_set_kernel_variant). The state is copied aside first and restored afterwards, so
   it is unchanged bit for bit. This call allocates a temporary copy of the radiation
   fields and synchronises; the choice is also remembered for later handles of the same
   grid shape and precision in this process. RHD_ECFL if chat dt_rad > K0 dx. */
int rhd_autotune(rhd_t* h, double chat, double dt_rad, int reps, int* variant, int* tile_rows,
                 int* zchunk);

/* ---- many independent solves advanced together (served form) ------------------------- */

typedef struct rhd_batch rhd_batch_t;

/* Create a batch that advances up to max_solves independent 3D handles together: every
   radiation Van Leer stage of all members goes out as one launch over a packed list of
   tiles (64 x tile_rows cells, zchunk planes; tile_rows 4, 8 or 16 in mixed precision,
   4 or 8 in FP64; in mixed precision the predictor's tiles are 4 rows by at most 11
   planes, as for a lone handle). hip_stream is a hipStream_t or NULL for an owned stream. */
int rhd_batch_create(void* hip_stream, int max_solves, int tile_rows, int zchunk,
                     rhd_batch_t** out);

/* Add a handle and the reduced speed of light it runs with. The handle must hold a state,
   be 3D, have the precision of the batch (the first member fixes it) and belong to no
   other batch; RHD_EINVAL otherwise, or when the batch is full. While it is a member its
   work runs on the batch's stream; on the handle itself only rhd_get_state,
   rhd_get_diagnostics, rhd_ledger and rhd_sync may be called (they wait for that stream).
   The batch's stream waits, on the device, for the work the handle's own stream holds; the
   host does not wait, except when the batch's tile lists must grow (device allocation),
   where it first waits for the batch's stream. */
int rhd_batch_add(rhd_batch_t* b, rhd_t* h, double chat);

/* Remove a member and give the handle its own stream back. That stream waits, on the
   device, for the batch's work enqueued so far; the host does not wait. */
int rhd_batch_remove(rhd_batch_t* b, rhd_t* h);

/* Advance every member by one gas step with its own CFL step and subcycle count
   (Sec. 3.1, Eqs. algorithm:gastimestep and algorithm:radtimestep): one synchronisation
   reads all v_max values; the exchange and gas step of each member follow; then the
   radiation subcycles of all members run over one packed list of tiles as rounds of two
   launches (predictor and corrector), round r covering the members with nsub > r; each
   member's correction and ledger close the step.
   A member's result does not depend, bit for bit, on which other solves share the batch
   or on the launch mode; it equals what rhd_step gives the handle alone to rounding (the
   kernels differ).
   nsub_out and dt_out (each NULL or room for rhd_batch_size() values, member order)
   receive each member's nsub and dt_gas. A member whose v_max is not finite and positive
   (RHD_ENONFINITE) or that needs more than 4096 subcycles (RHD_EINVAL) stops the call
   before anything is enqueued; nsub_out then holds -1 for that member and 0 for the
   others, so the caller can remove it and step again. Allocates nothing. */
int rhd_batch_step(rhd_batch_t* b, int* nsub_out, double* dt_out);

/* Launch mode of rhd_batch_step's radiation subcycles: 0, rounds of two launches (the
   only mode that runs). 1 asks for one persistent launch with per-member phase counters
   (blocks take tiles in order from a shared counter; a tile of a member's stage starts
   once that member's previous stage is complete). That launch is switched off, because
   it did not finish on the GPU: asking for it returns RHD_EINVAL and changes nothing. */
int rhd_batch_set_persistent(rhd_batch_t* b, int on);

/* Number of members. */
int rhd_batch_size(const rhd_batch_t* b);

/* Wait for the batch's stream. */
int rhd_batch_sync(rhd_batch_t* b);

/* Destroy the batch; members get their own streams back (they are not destroyed). */
void rhd_batch_destroy(rhd_batch_t* b);

/* Message of the last failure of a batch call (b may be NULL for rhd_batch_create). */
const char* rhd_batch_last_error(const rhd_batch_t* b);

/* ---- served form: independent solves submitted over time ------------------------------ */

/* A server owns a worker thread that solves independent 3D problems on the HIP device
   that was current at rhd_server_create. Requests wait in submission order; the worker
   admits the oldest ones while the sum of their rhd_footprint_bytes stays within the
   budget and at most max_slots run, and advances every running request one gas step per
   round through batches (rhd_batch_*, one per precision) with tiles of tile_rows x zchunk.
   Transfer threads work beside it (six for each direction): they create admitted
   requests' handles and upload their states, and copy finished requests' states to host
   memory and free their handles, so the batch keeps stepping meanwhile. A request leaves as soon as it has
   taken its steps: its state is copied to host memory, its device memory and slot are
   freed and the next requests are admitted. Every call
   below may come from any host thread. None of this is from the paper: it serves many
   solves of the paper's step (Sec. 3.1) on one device. */
typedef struct rhd_server rhd_server_t;

#define RHD_REQ_QUEUED     0  /* waiting for memory or a slot                               */
#define RHD_REQ_RUNNING    1
#define RHD_REQ_DONE       2  /* its steps taken; the final state waits for rhd_server_fetch */
#define RHD_REQ_FAILED     3  /* stopped with error `error` (state as computed, fetchable)   */
#define RHD_REQ_CANCELLED  4

typedef struct {
  int status;                 /* RHD_REQ_*                                                  */
  int error;                  /* RHD_* code of a failed request, else RHD_OK                */
  int steps_done;             /* gas steps taken                                            */
  long long zone_updates;     /* cells x radiation subcycles taken                          */
  double t_submit, t_start, t_done;  /* seconds on the server's steady clock since its
                                        creation; t_start / t_done are -1 until reached     */
} rhd_request_info;

typedef struct {
  long long submitted, completed, failed, cancelled, rejected;
  long long zone_updates;     /* over all requests                                          */
  long long rounds;           /* batch steps the worker took                                */
  long long bytes_in_use, peak_bytes;  /* sum of the running requests' footprints          */
  int running, queued, peak_running;
} rhd_server_stats;

/* Create a server. RHD_EINVAL for budget_bytes <= 0, max_slots < 1 or a tile shape the
   batches reject (tile_rows 4, 8 or 16; zchunk >= 1). On failure *out is NULL. */
int rhd_server_create(long long budget_bytes, int max_slots, int tile_rows, int zchunk,
                      rhd_server_t** out);

/* Launch mode of the server's batches (see rhd_batch_set_persistent): 0, rounds of two
   launches, the default and the only mode that runs; 1 returns RHD_EINVAL (the
   persistent launch is switched off). Only before the first submission (RHD_ESTATE
   after). */
int rhd_server_set_persistent(rhd_server_t* s, int on);

/* Queue a request: parameters and initial state as for rhd_create, rhd_set_state and
   rhd_set_emission (j may be NULL), then `steps` gas steps, each with the CFL step and
   subcycle count rhd_suggest_dt gives at the reduced speed of light chat. The host arrays
   are copied before the call returns. *id receives the request's id (ids count up from
   1). RHD_EINVAL for invalid parameters, a grid that is not 3D, a fixed face, steps < 1
   or chat <= 0;
   RHD_ENOMEM when the request's footprint alone exceeds the budget, so that it could
   never be admitted (nothing is queued then). */
int rhd_server_submit(rhd_server_t* s, const rhd_params* p, const double* rho,
                      const double* mom, const double* E, const double* Er, const double* Fr,
                      const double* kappaP, const double* kappaF, int kappa_scalar,
                      const double* j, int steps, double chat, long long* id);

/* Status and timing of a request, without waiting. RHD_EINVAL for an unknown id. */
int rhd_server_poll(rhd_server_t* s, long long id, rhd_request_info* info);

/* Wait until the request is done, failed or cancelled, then as rhd_server_poll.
   timeout_s < 0 waits without limit; RHD_ETIMEOUT when the time runs out first. */
int rhd_server_wait(rhd_server_t* s, long long id, double timeout_s, rhd_request_info* info);

/* Copy the final state of a finished request (host FP64 arrays as rhd_get_state; any may
   be NULL) and its diagnostics (may be NULL), then forget the request. Returns RHD_OK for
   a done request, the request's error for a failed one (the state is copied as computed),
   RHD_ESTATE for a queued, running or cancelled one, RHD_EINVAL for an unknown id. */
int rhd_server_fetch(rhd_server_t* s, long long id, double* rho, double* mom, double* E,
                     double* Er, double* Fr, rhd_diag* diag);

/* Cancel a request. A queued one is dropped at once; a running one leaves its batch
   before the next round, which frees its memory and slot; the other requests' results do
   not change. A finished request is forgotten. RHD_EINVAL for an unknown id. */
int rhd_server_cancel(rhd_server_t* s, long long id);

/* Counters of the server's life so far. */
int rhd_server_get_stats(rhd_server_t* s, rhd_server_stats* out);

/* Stop the worker after its current round, drop every request and free everything.
   No other call on this server may be in progress or follow. NULL is ignored. */
void rhd_server_destroy(rhd_server_t* s);

/* Message of the last failure of a call on this server or of its worker (s may be NULL
   for rhd_server_create). The text is copied for the calling thread: it stays valid
   until that thread's next call of this function. */
const char* rhd_server_last_error(const rhd_server_t* s);

/* Device bytes the handle holds (state, opacities, emission and scratch). The state and
   scratch buffers share one allocation, each rounded up to 4 KiB. */
long long rhd_device_bytes(const rhd_t* h);

/* Device bytes a handle with these parameters holds when created, before per-cell
   opacities or an emissivity are set; equal to rhd_device_bytes of such a handle. */
long long rhd_footprint_bytes(const rhd_params* p);

/* ---- radiation subcycles without allocation ------------------------------------------ */

/* Bytes of device scratch the allocation-free entry point below holds on each device it
   runs on: a file-scope device array of the library, kept until the process ends. */
#define RHD_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
   serving loops, harnesses that forbid allocation. It advances nsub radiation Van Leer
   subcycles of dt_gas/nsub each on caller-owned device arrays, with the gas frozen: the
   same kernels and arithmetic as the subcycles of rhd_step on a handle with the same
   parameters and default kernel choice, so the radiation state comes out the same bit
   for bit. It calls no hipMalloc, hipFree or allocating library routine: the half-step
   arrays and the clamp and floor counters live in the library's scratch array
   (RHD_NOALLOC_SCRATCH_BYTES per device, looked up on the first call on each device).
   Work is enqueued on hip_stream (a hipStream_t, or NULL for the null stream); no
   synchronisation.
   Arguments (device pointers of the current device; element type double, or float with
   RHD_PRECISION_MIXED; N = nx ny nz cells in the usual layout):
     p        -- parameters as for rhd_create; the exchange, gas and step-size fields are
                 ignored except theta_F, cfl, er_floor, the closure, RHD_BETA_TAU and
                 RHD_EXCHANGE_ABSORB_ONLY (kappa_P damping of E_r on each stage);
     Er, Fr   -- radiation state, N and 3N values, updated in place;
     rho      -- gas density, N values; mom -- gas momentum, 3N values, read only with
                 RHD_BETA_TAU (else may be NULL);
     kappaP, kappaF -- per-cell specific opacities (N each), or both NULL to use the
                 scalars kappaP_s, kappaF_s;
     j        -- emissivity, N values, or NULL.
   Errors: RHD_EINVAL for invalid parameters, RHD_OPACITY_LAW, fixed faces, NULL state
   arrays, nsub < 1, dt_gas or chat not finite and > 0, or a grid whose half-step arrays
   exceed the scratch (rhd_subcycles_noalloc_bytes(p) > RHD_NOALLOC_SCRATCH_BYTES: up to
   157^3 cells in mixed precision, 123^3 in FP64); RHD_ECFL as for rhd_step; RHD_EDEVICE
   if a launch fails. rhd_last_error(NULL) holds the message. Every call on one device
   shares the scratch array, so calls that overlap in time on one device (other streams,
   other host threads) race and give wrong results; serialise them. The counters are
   cleared at the start of each call and not reported. */
int rhd_subcycles_noalloc(const rhd_params* p, void* hip_stream, void* Er, void* Fr,
                          const void* rho, const void* mom, const void* kappaP,
                          const void* kappaF, double kappaP_s, double kappaF_s, const void* j,
                          double dt_gas, double chat, int nsub);

/* Scratch bytes rhd_subcycles_noalloc needs for these parameters (-1 if p is invalid). */
long long rhd_subcycles_noalloc_bytes(const rhd_params* p);

/* Free every device buffer and the owned stream. A batch member leaves its batch first
   (as with rhd_batch_remove). NULL is ignored. */
void rhd_destroy(rhd_t* h);

/* Message of the last failure on this handle (or of the last failed rhd_create when h
   is NULL). Never NULL. */
const char* rhd_last_error(const rhd_t* h);

#ifdef __cplusplus
}
#endif
#endif /* RHD_H */
