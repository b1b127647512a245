/*
 * vplbm.h -- C ABI of the MI355X (gfx950) volume-penalization lattice-Boltzmann
 * library: one D2Q9 multiple-relaxation-time time step with the penalization force
 * of a moving rigid disc, its force/torque and the rigid-body update.
 *
 * Method: Liberge & Beghein, "Fluid Structure Interaction modelling using Lattice
 * Boltzmann and Volume Penalization method" (arXiv 1905.05110):
 *   Sec. 2.1, Eqs. (1)-(2)      penalized Navier-Stokes, indicator chi of the solid;
 *   Sec. 2.2, Eqs. (8)-(22)     MRT lattice Boltzmann with a Guo source, the implicit
 *                               penalized velocity update (Eq. (22));
 *   Sec. 2.3, Eqs. (23)-(24)    rigid-body translation/rotation, solved by RK4;
 *   Algorithm 1                 order of one fluid-structure step.
 * The force on the body is the volume integral of the penalization force,
 * sum over nodes of rho chi/eta (u - u_s), instead of the momentum-exchange sum of
 * Eqs. (25)-(27).
 *
 * Conventions for every call:
 *   - Every function returns an int status (LBM_OK or a negative LBM_ERR_*); nothing
 *     is thrown across the ABI.  lbm_last_error(sim) gives a message valid until the
 *     next call on the same handle; lbm_last_error(NULL) gives the message of the last
 *     failed lbm_create on this thread.
 *   - Arguments are checked before any device call; a rejected call changes nothing.
 *   - lbm_step only enqueues work on the simulation's HIP stream and returns launch
 *     errors.  Errors during execution surface at the next synchronising call
 *     (lbm_sync, lbm_forces, lbm_fields, lbm_get_populations, lbm_save).
 *   - Host arrays are owned by the caller.  Device memory allocated by the library is
 *     freed by lbm_destroy; device memory passed in through lbm_opts.pop_buffers is
 *     owned by the caller and must outlive the simulation.
 *   - A handle must not be used by two threads at once; separate handles are
 *     independent.
 *   - Fields and population arrays on the host are FP64, [ny][nx] (x fastest) or
 *     [9][ny][nx], whatever the storage precision on the device.
 *   - Lattice: node (i, j) sits at x = i, y = j (lattice units, dx = dt = 1); domain
 *     walls sit half-way, at -1/2 and n - 1/2.  Directions: 0 rest, 1 E, 2 N, 3 W,
 *     4 S, 5 NE, 6 NW, 7 SW, 8 SE (Sec. 2.2, Eq. (10)).
 */
#ifndef VPLBM_H
#define VPLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sim lbm_sim; /* opaque, owned by the library */

enum {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,      /* invalid argument; nothing was done */
    LBM_ERR_ALLOC = -2,    /* device or host allocation failed */
    LBM_ERR_HIP = -3,      /* HIP runtime error (message in lbm_last_error) */
    LBM_ERR_UNSTABLE = -4, /* a non-positive or non-finite density/velocity was met */
    LBM_ERR_STATE = -5     /* call not valid in the current state */
};

/* Storage of the populations in device memory.  All forms store the offset
 * g = f - f_ref from a reference equilibrium (see lbm_opts.offset_ref); arithmetic is
 * FP64 for LBM_FP64 and FP32 otherwise; force/torque reductions and the rigid body
 * are always FP64.
 * LBM_FP16_OFS stores round-to-nearest-even(g * 2^k) as IEEE binary16 (k =
 * fp16_scale_log2); LBM_BF16_OFS stores round-to-nearest-even(g) as bfloat16. */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_OFS = 2, LBM_BF16_OFS = 3 };

/* Reference equilibrium of the stored offsets: INITIAL uses f_eq(1, u0) (the initial
 * or inflow state, so a uniform stream is stored as zeros); REST uses the rest-state
 * weights w_a = f_eq(1, 0); AUTO (the default) takes REST for the 16-bit storages and
 * INITIAL for FP32 and FP64.  With 16-bit storage the rest reference keeps the stored
 * magnitudes, hence the rounding, smallest where the flow is slow (near the body). */
enum { LBM_REF_AUTO = 0, LBM_REF_INITIAL = 1, LBM_REF_REST = 2 };

/* Store instructions for the populations: PLAIN keeps them in the caches (a grid whose
 * two buffers fit the 256 MB Infinity Cache then runs from it); NONTEMPORAL streams
 * them past the caches; AUTO picks NONTEMPORAL above 1 GiB of buffers. */
enum { LBM_STORE_AUTO = 0, LBM_STORE_PLAIN = 1, LBM_STORE_NONTEMPORAL = 2 };

/* Arrangement of the nine population arrays of a buffer (each row of a direction holds
 * pitch = nx rounded up to an odd multiple of 64 elements; the padding is never read or
 * written):
 *   ROWS    row-interleaved: row j of direction a at element (9 j + a) pitch, so that the
 *           three source rows and the destination row of a node lie close together;
 *   PLANES  one plane per direction, [9][ny][pitch] plus a small pad between planes;
 *   AUTO    ROWS when it fits, else PLANES.
 * Buffers may be of any size: the step addresses each tile's populations with 32-bit
 * offsets from bases at the tile's own rows, the other paths with 64-bit offsets.  The
 * 18 rows a tile reaches must span less than 4 GiB: ROWS takes up to 3.3 M columns in
 * FP64 (6.6 M in FP32, 13 M in 16-bit storage), PLANES nine times as many; lbm_create
 * refuses wider grids with LBM_ERR_ARG (and the adjoint, whose reverse step uses 32-bit
 * offsets from a direction's base, refuses grids whose direction arrays reach 4 GiB).
 * Both take lbm_pop_bytes() bytes; results are bitwise the same in either. */
enum { LBM_LAYOUT_AUTO = 0, LBM_LAYOUT_ROWS = 1, LBM_LAYOUT_PLANES = 2 };

/* Where the body state of a step is made final.  The tiles that meet the body write
 * partial FP64 force sums; the next step needs their total (and the rigid-body update it
 * drives) before it can place the body.
 *   TILES   every tile of the next step that meets the body adds all the slots itself
 *           (no extra launch; for a body over P tiles, P^2 slot reads per step);
 *   KERNEL  a one-workgroup launch after each step adds them once and writes the state;
 *   AUTO    KERNEL when the body's tiles number more than 512, else TILES.
 * Both add the slots in the same fixed order: results are bitwise the same. */
enum { LBM_FINALIZE_AUTO = 0, LBM_FINALIZE_TILES = 1, LBM_FINALIZE_KERNEL = 2 };

/* Collision operator.  MRT relaxes the moments of Eq. (9) at the rates of lbm_rates
 * (Eqs. (8), (16)); BGK (Sec. 2.2, Eqs. (11)-(12) with Guo's source) relaxes every
 * population at 1/tau = s_nu, which is MRT with all rates equal to s_nu: with it,
 * s_e, s_eps and s_q are ignored. */
enum { LBM_COLLIDE_MRT = 0, LBM_COLLIDE_BGK = 1 };

/* Boundary rule of one domain side (Sec. 3.1 for the channel set-up).
 *   PERIODIC  wrap around (both opposite sides must be periodic);
 *   WALL      no-slip half-way bounce-back;
 *   VELOCITY  half-way bounce-back of a wall moving at u_wall (inlet of Sec. 3.1):
 *             f_a = f~_opp(a) + 6 w_a (c_a . u_wall), wall density 1;
 *   SYMMETRY  free-slip specular reflection (u . n = 0);
 *   OUTFLOW   convective outflow df/dt + U_c df/dx = 0, implicit upwind in time
 *             (east side only).
 * At corners the west/east rule is applied first. */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1, LBM_BC_VELOCITY = 2, LBM_BC_SYMMETRY = 3,
       LBM_BC_OUTFLOW = 4 };
enum { LBM_WEST = 0, LBM_EAST = 1, LBM_SOUTH = 2, LBM_NORTH = 3 };

/* Body motion.  FIXED: pose constant (its velocities still enter u_s);
 * IMPOSED_SIN: y = imp_y0 + imp_amp sin(2 pi imp_freq t), t = steps since
 * lbm_set_body (shape of Sec. 3.1, Eq. (29)); FREE: Eqs. (23)-(24) by classical RK4
 * with unit step and the fluid force frozen over the step, for the degrees of freedom
 * set in free_mask (bit 0 x, bit 1 y, bit 2 theta), the others held; CONST_VEL: pose
 * advances by its constant velocities every step. */
enum { LBM_BODY_FIXED = 0, LBM_BODY_IMPOSED_SIN = 1, LBM_BODY_FREE = 2, LBM_BODY_CONST_VEL = 3 };

/* Load that drives a FREE body, and whether the momentum-exchange sum of Sec. 2.3,
 * Eqs. (25)-(27) is evaluated (it costs a pass over the body's tiles every step):
 *   LBM_FORCE_VP      the penalization force with the internal-momentum term (fh);
 *                     fmem and tmem are recorded as 0
 *   LBM_FORCE_MEM     the momentum-exchange force and torque (fmem, tmem)
 *   LBM_FORCE_VP_MEM  fh drives the body; fmem and tmem are recorded alongside */
enum { LBM_FORCE_VP = 0, LBM_FORCE_MEM = 1, LBM_FORCE_VP_MEM = 2 };

/* MRT relaxation rates of the non-conserved moments (Sec. 2.2, Eq. (16)):
 * s_e (energy), s_eps (energy square), s_q (heat fluxes), s_nu (stresses; 1/tau,
 * nu = (tau - 1/2)/3 by Eq. (6)).  Each must lie in (0, 2).  The rates of the
 * conserved moments do not change the result and are not inputs. */
typedef struct {
    double s_e, s_eps, s_q, s_nu;
} lbm_rates;

typedef struct {
    int bc[4];             /* LBM_BC_* for west, east, south, north */
    double u_wall[4][2];   /* wall velocity of each side (used by VELOCITY sides) */
    double u_conv;         /* convective velocity U_c of an OUTFLOW side, >= 0 */
    double g_fluid[2];     /* uniform body-force acceleration on the fluid */
    double rho0, u0[2];    /* initial state f = f_eq(rho0, u0) everywhere */
    int storage;           /* LBM_FP64 / LBM_FP32 / LBM_FP16_OFS / LBM_BF16_OFS */
    int fp16_scale_log2;   /* k of the FP16 offset scale 2^k, 0..14 (default 10) */
    int history_cap;       /* force records kept on the device between drains (default 65536) */
    int offset_ref;        /* LBM_REF_AUTO (default), LBM_REF_INITIAL or LBM_REF_REST */
    int rows_per_tile;     /* grid rows per lane of the step kernel: 1, 2, 4;
                              0 = default (1).  Each setting is deterministic; results of
                              different settings agree to rounding (kernel variants may
                              contract multiply-adds differently; FP64 force sums follow
                              the tile order). */
    int store_mode;        /* LBM_STORE_AUTO (default), _PLAIN or _NONTEMPORAL */
    void* hip_stream;      /* hipStream_t to run on; NULL: the library creates one */
    void* pop_buffers[2];  /* optional caller-owned device buffers of lbm_pop_bytes() each */
    int collision;         /* LBM_COLLIDE_MRT (default) or LBM_COLLIDE_BGK */
    int tile_width;        /* grid columns per tile of the step kernel: 0 = default
                              (256), 64, 256 or 512.  A tile of 256 or 512 columns is one
                              workgroup of as many threads, rows_per_tile rows high; a
                              tile of 64 columns is a 256-thread workgroup whose four
                              waves take four consecutive row groups, 4 rows_per_tile
                              rows high (narrow or ragged grids leave fewer idle lanes).
                              Like rows_per_tile a launch choice: results of different
                              settings agree to rounding (the FP64 force sums follow the
                              tile order). */
    int layout;            /* LBM_LAYOUT_AUTO (default), _ROWS or _PLANES */
    int finalize;          /* LBM_FINALIZE_AUTO (default), _TILES or _KERNEL */
} lbm_opts;

typedef struct {
    double radius, x, y, theta, vx, vy, omega; /* disc radius, pose and velocities at t = 0 */
    int mode;                                  /* LBM_BODY_* */
    unsigned free_mask;                        /* FREE: bit 0 x, bit 1 y, bit 2 theta */
    double mass, inertia;                      /* m and I of Eqs. (23)-(24) */
    double k[3], c[3], q0[3], f_ext[3];        /* stiffness, damping, rest pose, external load */
    double imp_amp, imp_freq, imp_y0;          /* IMPOSED_SIN: y = y0 + A sin(2 pi f t + phase),
                                                  t in steps since lbm_set_body; phase =
                                                  pi/2 gives the cosine law of Eq. (29) */
    double smooth_delta;                       /* 0: sharp chi (d^2 <= R^2); > 0: chi =
                                                  1/(1 + exp(2 (d - R)/delta)), 0 beyond
                                                  d - R > 20 delta, 1 below -20 delta */
    int internal_mass_correction;              /* 1: fh includes the internal-momentum
                                                  change (see lbm_force_rec) */
    double imp_phase;                          /* IMPOSED_SIN phase (radians) */
    int force_model;                           /* LBM_FORCE_* (default LBM_FORCE_VP) */
} lbm_body;

/* Per-step record, written on the device for every step. */
typedef struct {
    int64_t step;      /* index of the step */
    double fvp[2];     /* sum over nodes of rho chi/eta (u - u_s): force on the body */
    double tvp;        /* its torque about the body centre */
    double pin[3];     /* post-collision momentum and angular momentum of the fluid inside
                          the body: sum chi (j + G), sum chi r x (j + G) */
    double fh[2], th;  /* hydrodynamic force/torque, fvp + pin(n) - pin(n-1) when
                          internal_mass_correction is set (else fvp): for a sharp chi the
                          momentum streamed across the interface (the momentum-exchange
                          force of Eqs. (25)-(27)); FREE bodies are driven by it.  On the
                          first step after lbm_set_body, pin(n-1) is the pre-collision
                          momentum inside the body, sum chi j. */
    double q[3], v[3]; /* pose (x, y, theta) and velocities during this step */
    double fmem[2];    /* (LBM_FORCE_MEM, LBM_FORCE_VP_MEM; else 0) momentum-exchange
                          force of Eqs. (25)-(27): over the links from a
                          fluid node x_f to a solid node x_s = x_f + c_a (solid: d^2 <= R^2,
                          whatever the indicator mode), (c_a - u_G) f~_a(x_f) - (-c_a - u_G)
                          f~_abar(x_s), with x_G the crossing of the link and the circle
                          and u_G the rigid velocity there (post-collision populations) */
    double tmem;       /* its torque about the body centre, sum (x_G - X) x F */
} lbm_force_rec;

/* Fills o with defaults: periodic on all sides, rho0 = 1, u0 = 0, FP32 storage. */
void lbm_default_opts(lbm_opts* o);

/* Bytes of one population buffer (two are needed) for a grid and storage. */
size_t lbm_pop_bytes(int nx, int ny, int storage);

/* Creates a simulation on the current HIP device.  nx, ny >= 3; every rate in (0, 2);
 * eta > 0 (penalization factor of Eq. (1)); opts NULL means lbm_default_opts.
 * Periodic sides must come in opposite pairs; OUTFLOW only on the east side and then
 * nx >= 3.  On success *out receives the handle. */
int lbm_create(int nx, int ny, lbm_rates rates, double eta, const lbm_opts* opts,
               lbm_sim** out);

/* Sets (or replaces) the rigid disc; allowed before and between steps.  radius > 0,
 * mass > 0 and inertia > 0 for FREE bodies.  Resets the imposed-motion clock and the
 * internal-momentum history. */
int lbm_set_body(lbm_sim* sim, const lbm_body* body);

/* Removes the body (chi = 0 everywhere). */
int lbm_clear_body(lbm_sim* sim);

/* Enqueues n >= 0 time steps (Algorithm 1) on the simulation's stream. */
int lbm_step(lbm_sim* sim, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): enqueues n >= 0 steps exactly as
 * lbm_step does with graphs off (eager launches on the simulation's stream; bitwise the
 * same results and records), allocating nothing.  The step kernels' only scratch memory,
 * the body's partial force sums (12 FP64 per tile that meets the body), then lives in a
 * static array of the library (2 MiB per device, held until the process ends) instead
 * of the simulation's own.  LBM_ERR_ARG if the body spans more tiles than that holds
 * (10 922, counting one tile of slack each way).  The array is shared by every call on
 * a device: calls that overlap on one device (other host threads, other streams) race
 * and must not be made. */
int lbm_step_static(lbm_sim* sim, int64_t n);

/* Replays captured HIP graphs of k steps (k even, >= 2) inside lbm_step; k = 0 turns
 * graphs off.  Results are identical with and without graphs. */
int lbm_set_graph_steps(lbm_sim* sim, int k);

/* Waits for the stream; LBM_ERR_UNSTABLE if an unstable state was met. */
int lbm_sync(lbm_sim* sim);

/* Synchronises, then copies the records of the steps not yet drained, oldest first,
 * at most cap of them, into out; *n_out receives the count.  Records overwritten on
 * the device before being drained (more than history_cap pending) are skipped.  Steps
 * taken without a body have no record; setting a body on a simulation that has none
 * discards records still pending from an earlier body. */
int lbm_forces(lbm_sim* sim, lbm_force_rec* out, int64_t cap, int64_t* n_out);

/* Synchronises, then writes density and penalized velocity (Eq. (22)) of the current
 * state with the body at its current pose into host arrays of nx*ny doubles each.  The
 * first call of lbm_fields, lbm_set_populations or lbm_get_populations on a simulation
 * allocates its FP64 exchange buffer on the device (9 nx ny doubles, kept until
 * lbm_destroy); LBM_ERR_ALLOC if that fails. */
int lbm_fields(lbm_sim* sim, double* rho, double* ux, double* uy);

/* Debug access to the post-collision populations f (not offsets), host FP64
 * [9][ny][nx]; set is rounded to the storage precision.  See lbm_fields for the exchange
 * buffer. */
int lbm_set_populations(lbm_sim* sim, const double* f);
int lbm_get_populations(lbm_sim* sim, double* f);

/* Synchronises and returns the body pose and velocities (3 doubles each). */
int lbm_get_body_state(lbm_sim* sim, double* q, double* v);

/* Number of steps enqueued since creation. */
int64_t lbm_step_index(const lbm_sim* sim);

/* Enqueues n steps with a HIP event pair around every launch of the step kernel (the
 * grid-wide pull/collide kernel; the one-workgroup finalisation that follows it is
 * outside the pair), synchronises and returns the summed step-kernel time (ms) and the
 * time of the whole region (ms). */
int lbm_step_timed(lbm_sim* sim, int64_t n, double* kernel_ms, double* region_ms);

/* Chooses the launch configuration of the step kernel (rows per tile 1/2/4, plain or
 * nontemporal stores, 64, 256 or 512 columns per tile and, with a body, how its state is
 * finalized) by timing each candidate on a scratch simulation of the same grid, storage
 * and body, started from a copy of sim's current populations and outflow memory (call it
 * once the flow has developed: the uniform start state is exactly zero in offsets and
 * moves faster than a developed flow): two replays of a captured graph of trial_steps
 * steps (rounded down to even, at least 2), the faster counting.  It then applies to
 * sim (whose state is not touched) the fastest, or rather, of the candidates within 1 %
 * of the fastest, the one with the narrowest tiles (then the fewest rows per lane, plain
 * stores, the state finalized in the tiles): equal within the timing's spread, it reads
 * the fewest bytes.  cache_path (may be NULL) names a
 * JSON-lines file: a configuration found there for this device, storage and grid is
 * applied without timing, and a newly timed one is appended.  Outputs (each may be
 * NULL): the chosen rows, nt flag, and the measured time per step in microseconds (-1
 * when taken from the cache). */
int lbm_autotune(lbm_sim* sim, int trial_steps, const char* cache_path, int* rows_out,
                 int* nt_out, double* us_out);

/* The launch configuration in use (set at creation, by lbm_autotune, or for a batch
 * member by the batch): rows per tile, nontemporal-store flag, columns per tile.
 * Outputs may be NULL. */
int lbm_launch_config(const lbm_sim* sim, int* rows_out, int* nt_out, int* tile_width_out);

/* The population layout in use: LBM_LAYOUT_ROWS or LBM_LAYOUT_PLANES (never AUTO). */
int lbm_layout(const lbm_sim* sim, int* layout_out);

/* 1 if the body state is made final by a separate launch after each step (see
 * LBM_FINALIZE_*), else 0 (also without a body). */
int lbm_finalize_by_kernel(const lbm_sim* sim, int* kernel_out);

/* Serialises the full state (populations, outflow memory, body, step index) into a
 * host buffer; with buf NULL only *size_out is set.  lbm_load restores a state saved
 * from a simulation of the same grid and storage. */
int lbm_save(lbm_sim* sim, void* buf, size_t cap, size_t* size_out);
int lbm_load(lbm_sim* sim, const void* buf, size_t size);

/* ---- batches: many independent simulations advanced by one launch per step ----------
 * All simulations of a batch share the storage precision and the launch configuration
 * (rows per tile, store mode); each keeps its own grid, rates, boundaries, body,
 * buffers and FP64 reductions, so a simulation inside a batch computes bitwise the same
 * as alone with the same configuration.  One launch per step covers every tile of every
 * simulation, in an order (schedule) chosen at creation or by lbm_batch_autotune:
 *   GIVEN          simulation by simulation, in the order given;
 *   LARGEST_FIRST  simulation by simulation, largest grid first (default);
 *   INTERLEAVED    one row of tiles from each simulation in turn. */
typedef struct lbm_batch lbm_batch;
enum { LBM_ORDER_GIVEN = 0, LBM_ORDER_LARGEST_FIRST = 1, LBM_ORDER_INTERLEAVED = 2 };

typedef struct {
    int nx, ny;
    lbm_rates rates;
    double eta;
    const lbm_opts* opts;  /* may be NULL; its storage, stream, buffers and launch fields are
                              replaced by the batch's */
    const lbm_body* body;  /* may be NULL (no body) */
} lbm_batch_desc;

typedef struct {
    int storage;        /* LBM_FP64 / LBM_FP32 / LBM_FP16_OFS / LBM_BF16_OFS */
    int rows_per_tile;  /* 0 (default: 1), 1, 2 or 4 */
    int store_mode;     /* LBM_STORE_* */
    int order;          /* LBM_ORDER_* */
    void* hip_stream;   /* NULL: the library creates one */
    int tile_width;     /* 0 (default: 256), 64, 256 or 512 (see lbm_opts) */
    int layout;         /* LBM_LAYOUT_AUTO: each member's own opts->layout; else every
                           member takes this one */
    int finalize;       /* LBM_FINALIZE_AUTO: each member's own opts->finalize; else every
                           member takes this one (the members that finalize by kernel share
                           one launch per step) */
} lbm_batch_opts;

void lbm_default_batch_opts(lbm_batch_opts* o);

/* Creates n >= 1 simulations (each argument checked as by lbm_create and lbm_set_body).
 * On failure nothing is left allocated and lbm_batch_last_error(NULL) tells why. */
int lbm_batch_create(int n, const lbm_batch_desc* descs, const lbm_batch_opts* opts,
                     lbm_batch** out);

/* Enqueues n steps of every simulation (one kernel launch per step, or captured graphs
 * of k steps after lbm_batch_set_graph_steps(k), k even). */
int lbm_batch_step(lbm_batch* batch, int64_t n);
int lbm_batch_set_graph_steps(lbm_batch* batch, int k);

/* Waits for the batch; LBM_ERR_UNSTABLE if any simulation met an unstable state. */
int lbm_batch_sync(lbm_batch* batch);

/* Handle of member i, owned by the batch.  It serves lbm_forces, lbm_fields,
 * lbm_get_body_state, lbm_get/set_populations, lbm_set/clear_body, lbm_sync, lbm_save,
 * lbm_step_index; lbm_step, lbm_step_timed, lbm_set_graph_steps, lbm_autotune, lbm_load
 * and lbm_destroy return LBM_ERR_STATE on it. */
int lbm_batch_sim(lbm_batch* batch, int i, lbm_sim** out);
int lbm_batch_size(const lbm_batch* batch);

/* Sets the launch configuration: rows 1/2/4, LBM_STORE_PLAIN or _NONTEMPORAL, order
 * (the columns per tile stay as they are). */
int lbm_batch_configure(lbm_batch* batch, int rows, int store_mode, int order);

/* Chooses rows, store mode, columns per tile, order and (with bodies) how the body
 * states are finalized by timing each candidate on a scratch copy of the batch started
 * from the members' current states (as lbm_autotune: the faster of two replays of a
 * captured graph of trial_steps steps; rows, store mode and columns per tile by the
 * near-tie rule of lbm_autotune, then the order and the finalization by the faster),
 * then applies them (members' states are not touched; lbm_launch_config and
 * lbm_finalize_by_kernel on a member report the choice).
 * Outputs may be NULL; us_out is the time per batch step in microseconds. */
int lbm_batch_autotune(lbm_batch* batch, int trial_steps, int* rows_out, int* nt_out,
                       int* order_out, double* us_out);

/* The schedule order in use (LBM_ORDER_*). */
int lbm_batch_order(const lbm_batch* batch, int* order_out);

int lbm_batch_destroy(lbm_batch* batch);
const char* lbm_batch_last_error(const lbm_batch* batch);

/* ---- adjoint: gradients of the time-integrated penalization force --------------------
 * For a body held at a fixed pose with rigid velocity (V, Omega) (lbm_body with mode
 * LBM_BODY_FIXED), the objective
 *     J = sum_{n < N} ( w_x F_vp,x(n) + w_y F_vp,y(n) )
 * (F_vp the penalization force of step n, lbm_force_rec.fvp; w = 1 / (N rho0 U0^2 D / 2)
 * makes J the time-averaged drag coefficient) is differentiated in reverse mode through
 * the N steps (Sec. 2.2 step, Sec. 2.1 indicator): dJ/dchi at every node (the indicator
 * taken as a free field), dJ/d(X, Y) (through the smoothed indicator of lbm_body
 * smooth_delta > 0 and through u_s; a sharp indicator contributes through u_s only) and
 * dJ/d(V_x, V_y, Omega).  The forward run keeps a checkpoint every K steps; the backward
 * run recomputes each segment of K steps from its checkpoint and sweeps it in reverse.
 * Device memory: about (N/K + K + 8) population buffers (lbm_pop_bytes).
 * FP64 and FP32 storage (arithmetic in the storage precision). */
typedef struct lbm_adjoint lbm_adjoint;

typedef struct {
    int64_t steps;         /* N >= 1, a multiple of checkpoint_every */
    int checkpoint_every;  /* K >= 2, even */
    double weight_fx;      /* w_x */
    double weight_fy;      /* w_y */
    int use_graphs;        /* 1: segments run as captured HIP graphs; 0: eager launches */
} lbm_adjoint_opts;

/* N = 4000, K = 100, w = (1, 0), graphs on */
void lbm_default_adjoint_opts(lbm_adjoint_opts* o);

/* Creates the simulation (arguments as lbm_create and lbm_set_body; opts may be NULL)
 * and the adjoint buffers.  The initial state is the uniform equilibrium (rho0, u0). */
int lbm_adjoint_create(int nx, int ny, lbm_rates rates, double eta, const lbm_opts* opts,
                       const lbm_body* body, const lbm_adjoint_opts* aopts, lbm_adjoint** out);

/* Moves the body (mode FIXED); the next forward run starts again from the initial state. */
int lbm_adjoint_set_body(lbm_adjoint* adj, const lbm_body* body);

/* Adds a field to the body's indicator in the forward run: chi(i, j) = the disc's chi
 * + field[j][i] at every step (the additive indicator of a smoothed chi; dJ/dchi of
 * lbm_adjoint_gradient is the derivative with respect to it).  field is FP64 [ny][nx]
 * host memory, zero outside the body's box (the nodes within the disc's reach plus one
 * of its centre, where its own indicator may vary), else LBM_ERR_ARG; NULL removes it.
 * lbm_adjoint_set_body removes it too (the box moves with the body).  It takes effect
 * at the next lbm_adjoint_forward. */
int lbm_adjoint_set_chi_add(lbm_adjoint* adj, const double* field);

/* Initial state of the forward run: post-collision populations [9][ny][nx] and the
 * outflow memory [3][ny] (directions 3, 6, 7), FP64 host arrays; NULL restores the
 * uniform equilibrium for that part. */
int lbm_adjoint_set_initial(lbm_adjoint* adj, const double* f, const double* outlet);

/* Runs the N forward steps from the initial state, keeping the checkpoints; *J receives
 * the objective (FP64 sum of the per-step records in step order).  Synchronous. */
int lbm_adjoint_forward(lbm_adjoint* adj, double* J);

/* Records of the last forward run (up to cap, oldest first). */
int lbm_adjoint_forces(lbm_adjoint* adj, lbm_force_rec* out, int64_t cap, int64_t* n_out);

/* Reverse sweep over the last forward run.  Synchronous.  LBM_ERR_STATE without one. */
int lbm_adjoint_backward(lbm_adjoint* adj);

/* Gradients of the last backward run: dJ_dchi [ny][nx] (may be NULL), dJ_dpos (X, Y),
 * dJ_dvel (V_x, V_y, Omega); FP64 host arrays. */
int lbm_adjoint_gradient(lbm_adjoint* adj, double* dJ_dchi, double* dJ_dpos, double* dJ_dvel);

/* Measurement: average duration (microseconds, HIP events) of reps launches of the
 * adjoint step kernel and of the forward step kernel on the segment store.  Overwrites
 * the accumulators: run lbm_adjoint_backward again before reading gradients. */
int lbm_adjoint_time_kernels(lbm_adjoint* adj, int reps, double* adjoint_us, double* step_us);

int lbm_adjoint_destroy(lbm_adjoint* adj);
const char* lbm_adjoint_last_error(const lbm_adjoint* adj);

/* Frees everything the library allocated for the simulation. */
int lbm_destroy(lbm_sim* sim);

const char* lbm_last_error(const lbm_sim* sim);

#ifdef __cplusplus
}
#endif

#endif /* VPLBM_H */
