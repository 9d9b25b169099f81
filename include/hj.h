/*
 * hj.h -- C ABI of the MI355X (gfx950) Hamilton-Jacobi reachability library.
 *
 * The library computes the Backward Reachable Tube (BRT) of a 4D car
 * (x, y, v, theta) on a grid by time-stepping the HJ variational inequality
 * of arXiv 2012.04011 (eq (4)): one-sided derivatives (eq (5), or second-order
 * ENO), a Lax-Friedrichs Hamiltonian with the optimal bang-bang control and
 * disturbance plus dissipation, forward Euler (Algorithm 2) or two-stage TVD
 * Runge-Kutta, a CFL step from a max-reduction of the dissipation
 * coefficients (Algorithm 1, step-bound lines), and the clamp V = min(V0, V)
 * (Algorithm 2, end of the loop body).  The BRT is {z : V(z) <= 0}
 * (section "Hamilton-Jacobi Reachability Analysis").
 *
 * Conventions for every function:
 *   - Every function returns hj_status; nothing throws across the ABI.  On
 *     failure a message is available from hj_last_error() (thread-local), and
 *     the handle is unchanged: all arguments are validated before any device
 *     work is enqueued.
 *   - External array layout: C order [Nx][Ny][Nv][Ntheta], theta fastest --
 *     the paper's 4D array V[N1][N2][N3][N4].  Element type per `dtype`
 *     (HJ_F32 or HJ_F64); location per `where` (HJ_HOST or HJ_DEVICE; device
 *     pointers must be on the handle's device).
 *   - Ownership: inputs are copied during the call and stay the caller's.
 *     Device buffers allocated by hj_grid_create belong to the handle until
 *     hj_grid_destroy.
 *   - Streams: all device work is enqueued in order on the stream given to
 *     hj_grid_create (borrowed; NULL = the device's null stream).  Calls that
 *     return data to host memory synchronise that stream; the rest return
 *     before the GPU finishes.  Device outputs are ready in stream order.
 *   - Threads: one host thread per handle at a time; different handles may
 *     be used concurrently.
 */
#ifndef HJ_H
#define HJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HJ_OK = 0,
  HJ_ERR_INVALID_ARG = 1,   /* a null pointer, bad size, range or enum value */
  HJ_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  HJ_ERR_DEVICE = 3,        /* a HIP call failed (message names it) */
  HJ_ERR_NOT_READY = 4,     /* no target set yet */
  HJ_ERR_NONFINITE = 5,     /* NaN or infinity in an input array */
  HJ_ERR_UNSUPPORTED = 6    /* valid request this build does not implement */
} hj_status;

/* enum values used in the descriptors */
enum { HJ_F32 = 0, HJ_F64 = 1 };                      /* dtype / precision */
enum { HJ_HOST = 0, HJ_DEVICE = 1 };                  /* where an array lives */
enum { HJ_DYN_CAR4D = 0, HJ_DYN_DRIFT_INPUT = 1, HJ_DYN_CAR4D_STEER = 2 }; /* dynamics kind */
enum { HJ_UPWIND1 = 0, HJ_ENO2 = 1 };                 /* derivative scheme */
enum { HJ_EULER = 0, HJ_TVD_RK2 = 1 };                /* integrator */
enum { HJ_CLAMP_NONE = 0, HJ_CLAMP_MIN_V0 = 1 };      /* target clamp */
enum { HJ_NORM_BOX = 0, HJ_NORM_BALL = 1 };           /* test input set norm */
enum { HJ_INPUT_MAXIMIZES = 0, HJ_INPUT_MINIMIZES = 1 };

typedef struct hj_grid hj_grid; /* opaque, library-owned */

/*
 * Grid (section "Basic Numerical Solution": N_d nodes on axis d).  Axes are
 * x, y, v, theta.  An ordinary axis has n[d] >= 3 nodes including both ends,
 * x_i = lo + i (hi - lo) / (n - 1).  A periodic axis (bit d of
 * periodic_mask) has n[d] >= 3 nodes over one period hi - lo,
 * x_i = lo + i (hi - lo) / n.  hi > lo.  The total node count may not exceed
 * 2^31 - 1.
 */
typedef struct {
  int32_t n[4];
  double lo[4], hi[4];
  uint32_t periodic_mask;
} hj_grid_desc;

/*
 * Dynamics.
 * HJ_DYN_CAR4D: x' = v cos(theta) + d_x, y' = v sin(theta) + d_y, v' = a,
 *   theta' = w.  Control |a| <= a_max, |w| <= w_max maximises grad(V).f;
 *   disturbance |d_x| <= d_max[0], |d_y| <= d_max[1] minimises it (eq (3),
 *   eq (4); the paper's car, eq (6), with the steering term replaced by a
 *   bounded turn rate).  Axis 2 must be v and axis 3 theta.
 * HJ_DYN_CAR4D_STEER: the paper's car exactly (eq (6)): as HJ_DYN_CAR4D but
 *   theta' = v tan(delta) / L with the steering angle |delta| <= steer_max
 *   (radians, < pi/2) and wheelbase L = wheelbase > 0 (the experiment:
 *   a_max 1.5, steer_max pi/18, L 0.3 m); w_max is unused.
 * HJ_DYN_DRIFT_INPUT (closed-form checks): z' = drift + u, u nonzero only on
 *   the axes in in_axes_mask, |u| <= in_speed in the box (per axis) or
 *   Euclidean-ball norm (in_norm); the input maximises or minimises
 *   (in_role).
 * All bounds must be finite and >= 0.
 */
typedef struct {
  int32_t kind;
  double a_max, w_max, d_max[2];
  double drift[4], in_speed;
  uint32_t in_axes_mask;
  int32_t in_norm, in_role;
  double steer_max, wheelbase;
} hj_dynamics_desc;

/*
 * Scheme.  deriv: HJ_UPWIND1 (eq (5)) or HJ_ENO2; integrator: HJ_EULER
 * (Algorithm 2) or HJ_TVD_RK2; precision: HJ_F32 or HJ_F64 storage and
 * arithmetic of the time step (the CFL reduction is always FP64); clamp:
 * HJ_CLAMP_MIN_V0 applies V = min(V0, V) once per full step; cfl in (0, 1].
 * alpha_mode: HJ_ALPHA_STATE (default): the dissipation coefficient
 * alpha_d(z) bounds |f_d| over every input, fixed per grid, one CFL step
 * for the whole solve.  HJ_ALPHA_DERIV_RANGE (Algorithm 1, the general
 * Lax-Friedrichs scheme): every step first finds, per axis, the smallest
 * and largest central derivative D_d V = (D+ V + D- V) / 2 (eq (5); with
 * ENO2 the average of its one-sided derivatives) over the grid's nodes,
 * takes alpha_d(z) = max |dH/dp_d| over that box of gradients and
 * dt = cfl / sum_d(alpha_d^max / dx_d), the last step shortened to the
 * horizon; both TVD-RK2 stages use the step's alpha (the range pass runs on
 * the stage kernel's own traversal where the LDS plane kernel runs the
 * grid).  HJ_ALPHA_DERIV_RANGE_ONESIDED: the same with the box spanned by
 * both one-sided derivatives of every node (the textbook global
 * Lax-Friedrichs bound, monotone over every pair of one-sided values on the
 * grid; never smaller than the central box).  Both need a host round trip
 * per step; batches, servers and the convergence mode reject them.
 */
enum { HJ_ALPHA_STATE = 0, HJ_ALPHA_DERIV_RANGE = 1, HJ_ALPHA_DERIV_RANGE_ONESIDED = 2 };

typedef struct {
  int32_t deriv, integrator, precision, clamp;
  int32_t alpha_mode;
  int32_t reserved; /* 0 */
  double cfl;
} hj_scheme_desc;

/* What a solve did: steps taken, the CFL step, the shortened last step and
 * the time reached (= the horizon). */
typedef struct {
  int64_t steps;
  double dt, dt_last, t_final;
} hj_solve_info;

/* Device-side timing of the time loop (HIP events recorded on the handle's
 * stream around the step kernels of each solve while profiling is on). */
typedef struct {
  int64_t solves;         /* solves timed */
  int64_t step_launches;  /* step-kernel launches inside the timed loops */
  double loop_ms;         /* summed event time of the timed loops */
} hj_profile;

/*
 * Create a grid handle: validates the descriptors, allocates the device
 * buffers (target V0, value V and the step's stage buffers, N values each in
 * the scheme's precision) and builds the per-(v, theta) coefficient table on
 * the host in FP64 (section "Indexed Processing Element": state vectors and
 * cos/sin kept in a lookup table).  hip_stream is a hipStream_t (borrowed,
 * must outlive the handle) or NULL.  *out receives the handle.
 * Errors: HJ_ERR_INVALID_ARG, HJ_ERR_OUT_OF_MEMORY, HJ_ERR_DEVICE.
 */
hj_status hj_grid_create(const hj_grid_desc *grid, const hj_dynamics_desc *dyn,
                         const hj_scheme_desc *scheme, void *hip_stream, hj_grid **out);

/* Free every buffer of the handle (after synchronising its stream).  NULL is
 * accepted and ignored. */
hj_status hj_grid_destroy(hj_grid *g);

/*
 * Set the target V0 = l(z) from a caller array (eq (4): V(z, 0) = l(z); the
 * target set is {V0 <= 0}).  Also sets V := V0 and the time to 0.  v0 holds N
 * values of `dtype` at `where` in the external layout.  Non-finite values are
 * rejected (HJ_ERR_NONFINITE) and leave the handle unchanged.
 */
hj_status hj_set_target(hj_grid *g, const void *v0, int32_t dtype, int32_t where);

/*
 * Set the target to a union of m >= 1 cylinders in (x, y) (eq (7), minimum
 * over obstacles): V0 = min_o(sqrt((x - cx_o)^2 + (y - cy_o)^2) - r_o), the
 * same for every (v, theta); computed on the GPU in the scheme's precision.
 * cx, cy, r are host arrays of m finite doubles, r >= 0.  Also sets V := V0
 * and the time to 0.  Requires axes 0 and 1 to be x and y.
 */
hj_status hj_set_target_cylinders(hj_grid *g, const double *cx, const double *cy, const double *r,
                                  int32_t m);

/*
 * Fixed-horizon BRT solve: V := V0, then n = ceil(T / dt) full steps with the
 * CFL step dt (the last one shortened to T - (n - 1) dt), each step followed
 * by the clamp if enabled.  T >= 0 (T = 0: no step).  The first call on a
 * handle runs the CFL reduction and caches dt (the dissipation coefficients
 * depend on the grid only).  Returns before the GPU finishes; *info (may be
 * NULL) is filled on return.  Errors: HJ_ERR_NOT_READY without a target.
 */
hj_status hj_solve_brt(hj_grid *g, double horizon, hj_solve_info *info);

/*
 * One full time step (Euler, or both TVD-RK2 stages) from the current V,
 * followed by the clamp if enabled.  dt > 0 is used as given; dt <= 0 takes
 * the cached CFL step.  *dt_taken (may be NULL) receives the step used.
 */
hj_status hj_step(hj_grid *g, double dt, double *dt_taken);

/* The CFL step dt = cfl / sum_d(alpha_d^max / dx_d) in FP64 (a max-reduction
 * on the GPU over the dissipation coefficients of every node); a zero sum
 * returns +infinity.  Synchronises. */
hj_status hj_get_cfl_dt(hj_grid *g, double *dt);

/* The per-axis maxima alpha_d^max behind hj_get_cfl_dt (4 doubles). */
hj_status hj_get_alpha_max(hj_grid *g, double alpha_max[4]);

/* Copy the current V (or, for hj_get_target, V0) out in the external layout
 * as `dtype` at `where`.  HJ_HOST synchronises the stream. */
hj_status hj_get_value(hj_grid *g, void *out, int32_t dtype, int32_t where);
hj_status hj_get_target(hj_grid *g, void *out, int32_t dtype, int32_t where);

/* Replace the current V (checkpoint resume at a step boundary); V0 is kept.
 * Non-finite values are rejected. */
hj_status hj_set_value(hj_grid *g, const void *v, int32_t dtype, int32_t where);

/* Number of grid points N of the handle. */
hj_status hj_get_num_points(hj_grid *g, int64_t *n);

/* Turn the step-loop event timing on (1) or off (0); turning it on resets the
 * counters. */
hj_status hj_set_profiling(hj_grid *g, int32_t enable);

/* Read the step-loop timing (synchronises the stream). */
hj_status hj_get_profile(hj_grid *g, hj_profile *out);

/* Convergence mode (Algorithms 1 and 2: "compute the HJ PDE until it
 * converges").  V := V0, then steps of the CFL step while the largest change
 * of a step, eps = max over nodes |V_{t+1} - V_t|, is at or above threshold
 * (the printed test is inverted; read as: stop once eps < threshold), at
 * most max_steps steps (>= 1).  The stop test runs on the device after every
 * step (with the LDS plane kernel, eps is folded into the step's last stage;
 * otherwise a pass over V_t and V_t+1 computes it); the host looks at it
 * every 32 steps, and steps enqueued past the stop do nothing.  Synchronises.  A grid on which nothing moves takes
 * steps of one time unit. */
typedef struct {
  int64_t steps;     /* steps taken */
  int32_t converged; /* 1: eps < threshold stopped it, 0: max_steps did */
  int32_t reserved;
  double dt;         /* the step */
  double eps_last;   /* eps of the last step taken */
} hj_converge_info;

hj_status hj_solve_converge(hj_grid *g, double threshold, int64_t max_steps, hj_converge_info *info);

/* Optimal control at m arbitrary states (eq (9), applied by the paper's
 * safety controller when eq (8) V < 0.15 holds): grad V and V at each state
 * from multilinear interpolation over its grid cell of the nodal
 * central-difference gradient (one-sided at the ends of open axes, wrapped
 * on theta) and of V; states outside an open axis are clamped to it.
 * states: m x 4 (x, y, v, theta) FP64; controls: m x 2, (a, w) for
 * HJ_DYN_CAR4D or (a, delta) for HJ_DYN_CAR4D_STEER, bang-bang with ties
 * (zero gradient) to the + bound; values: m (may be NULL).  All three on the
 * host (synchronises) or all on the device (stream-ordered), per `where`.
 * Computed in FP64 from the current V.  HJ_ERR_UNSUPPORTED for the test
 * dynamics. */
hj_status hj_optimal_control(hj_grid *g, const double *states, int64_t m, int32_t where, double *controls,
                             double *values);

/* The control query of hj_optimal_control (same arguments, same kernel,
 * the same results) for callers that cannot allocate device memory: a
 * safety controller's loop that queries every tick, code under HIP graph
 * capture, harnesses that forbid allocation.  hj_optimal_control grows a
 * device staging buffer for host arrays (hipMalloc / hipFree inside the
 * call); this variant allocates nothing: host arrays pass through one
 * fixed device array of HJ_NOALLOC_MAX_STATES states (7 doubles each,
 * 3.5 MiB), which each device holds from its first hj_grid_create until
 * the process ends, and device arrays are used in place.  m above
 * HJ_NOALLOC_MAX_STATES is HJ_ERR_INVALID_ARG.  Every call on a device
 * shares that array (each call writes all of it that it reads), so calls
 * that overlap on one device -- from several host threads, or on handles
 * with different streams -- race and must be serialised by the caller. */
#define HJ_NOALLOC_MAX_STATES 65536
hj_status hj_optimal_control_noalloc(hj_grid *g, const double *states, int64_t m, int32_t where,
                                     double *controls, double *values);

/* How the time step runs on this handle.  kernel: 2 = LDS plane kernel, 1 =
 * streaming kernel, 0 = one-thread-per-node kernel (chosen by grid shape,
 * then by hj_autotune).  x_chunks: how many pieces each x sweep is split
 * into.  target_xy: 1 if the target is constant over (v, theta) (set by
 * hj_set_target_cylinders) and the clamp reads an Nx*Ny table instead of
 * the 4D V0.  plane_segments: with the plane kernel, how many blocks share
 * one (v, theta) plane (split along v when it has more than 768 runs of
 * theta nodes); 0 with the other kernels.  solve_graph: 1 if hj_solve_brt
 * replays its time loop as a captured HIP graph (grids of at most 64 MiB per
 * array, or as HJ_SOLVE_GRAPH=0/1 forces; bitwise the same result).
 * theta_run: theta nodes per thread of the stage kernel (4, 3, 2 or 1; the
 * plane kernel takes runs of 3 in FP32 where they pack a whole plane into
 * fuller waves, by an estimate or by hj_autotune).  span_blocks: 0 when
 * the plane kernel cuts each y row's x sweep into x_chunks pieces; else the
 * number of blocks that share all rows' x planes equally in row-major order
 * (so that every compute unit gets the same work; chosen by hj_autotune).
 * plane_rows: y rows per plane-kernel block, 1, or 2 where two neighbouring
 * rows share a block (each row's threads then load only their outer y
 * neighbours and read the inner ones from LDS; chosen by hj_autotune or
 * HJ_PLANE_ROWS=2); 0 with the other kernels.  reserved: 0.
 * bytes_per_point_step: algorithmic
 * HBM bytes one full step moves per grid node in this mode (each array read
 * once and written once per stage). */
typedef struct {
  int32_t kernel, x_chunks, target_xy, autotuned;
  int32_t plane_segments, solve_graph;
  int32_t theta_run, span_blocks;
  int32_t plane_rows, reserved;
  double bytes_per_point_step;
} hj_launch_info;

hj_status hj_get_launch_info(hj_grid *g, hj_launch_info *out);

/* Time the candidate launch configurations (stage kernel that fits the
 * shape, the plane kernel's theta runs and one- or two-row blocks, x-chunk
 * counts 1..8, 10, 12, 16) on the handle's current buffers, time the three
 * fastest again in three alternating rounds and keep the fastest of those; a
 * few tens of milliseconds, synchronises.  The result of a solve does
 * not depend on the choice (every candidate evaluates each node with the
 * same arithmetic).  hj_solve_brt calls it on first use unless disabled by
 * hj_set_autotune(g, 0) or fixed by the HJ_X_CHUNKS / HJ_STAGE_KERNEL
 * environment variables.  Requires a target (HJ_ERR_NOT_READY).
 * Environment (for tests and measurements; read when a handle is created,
 * HJ_AUTOTUNE_VERBOSE when it autotunes):
 * HJ_STAGE_KERNEL=stream|generic forces a stage kernel; HJ_X_CHUNKS=n fixes
 * the x chunks; HJ_PLANE_RUN=3 or =the default run fixes the plane kernel's
 * theta run (where it fits); HJ_PLANE_SPAN=b shares all row-planes among b
 * plane-kernel blocks; HJ_PLANE_ROWS=1|2 keeps one-row or two-row plane
 * blocks (two-row blocks where a layout fits; the autotuner then times only
 * those); HJ_PLANE_VSEG=r splits the plane kernel's (v, theta) plane
 * into segments of at most r v rows (r >= 4) even when it fits one block;
 * HJ_AUTOTUNE_VERBOSE prints each candidate's time to stderr. */
hj_status hj_autotune(hj_grid *g);
hj_status hj_set_autotune(hj_grid *g, int32_t enable);

/* ---- Batched solves ------------------------------------------------------
 * Many independent BRT re-solves (different grids, obstacle sets and
 * horizons) run together on one device.  The paper solves one grid at a
 * time; a batch instance computes exactly what hj_solve_brt computes for its
 * handle (bitwise the same V), since every node's update depends only on the
 * previous step of its own grid (Algorithm 2, one sweep per step). */
typedef struct hj_batch hj_batch;

enum {
  HJ_BATCH_LAUNCHES = 0,   /* one launch per (step, stage) over every instance still running */
  HJ_BATCH_GRAPH = 1,      /* the same launches, captured once as a hipGraph and replayed */
  HJ_BATCH_PERSISTENT = 2, /* one persistent launch for the whole batch (work queue) */
  HJ_BATCH_STREAMS = 3     /* each instance's own single-grid solve, on 4 concurrent private streams */
};

typedef struct {
  int32_t m;                  /* instances */
  int32_t x_planes;           /* x planes per tile (streaming tile = 256 runs of theta nodes x x_planes;
                                 plane block = one y row's (v, theta) plane x x_planes), for the kernel
                                 of the last solve */
  int32_t persistent_blocks;  /* blocks of the last persistent launch */
  int32_t graph_nodes;        /* kernel nodes of the cached graph (0: none) */
  int64_t tiles_per_sweep;    /* tiles of one stage over all instances */
  int64_t work_items;         /* tiles over all stages of the last solve (0 after a streams-mode solve) */
  int64_t points;             /* grid nodes over all instances */
  int32_t plane_kernel;       /* 1: the last solve's launches ran the batched plane kernel */
  int32_t classes;            /* launch classes of the last solve (plane-kernel block sizes and the
                                 streaming tiles), each class's launches on a lane of its own */
} hj_batch_info;

/* Group m (1..256) grid handles.  They must share precision, derivative
 * scheme, integrator, device and stream, and have a periodic theta axis;
 * grids, dynamics, obstacle sets and clamp may differ.  The handles stay
 * owned by the caller and must outlive the batch; while a batch call runs,
 * no other call may use them.  Errors: HJ_ERR_INVALID_ARG (null, repeated
 * handle, m out of range), HJ_ERR_UNSUPPORTED (mixed schemes, streams or a
 * non-periodic theta). */
hj_status hj_batch_create(hj_grid *const *grids, int32_t m, hj_batch **out);
/* Launch- and graph-mode solves run the batched plane kernel (each
 * instance's blocks hold a y row's (v, theta) plane in LDS, as the
 * single-grid plane kernel) for the instances whose plane fits one of its
 * blocks of at most 768 work-items with runs of two or more theta nodes, and
 * the streaming tiles for the others; the persistent mode always runs
 * streaming tiles.  Launches are grouped into classes: plane blocks of 1-2,
 * 3-4 and 5-12 waves, and the streaming tiles; with more than one class,
 * each runs on a private stream forked from the batch stream and joined back
 * into it.  HJ_BATCH_KERNEL=stream (read at create) keeps every instance on
 * the streaming tiles. */
hj_status hj_batch_destroy(hj_batch *b);

/* Solve instance j over horizons[j] (finite, >= 0; m entries) from its
 * current target, exactly as hj_solve_brt(grids[j], horizons[j]) would, and
 * leave V in its handle; infos (m entries) may be NULL.  Launch-mode and
 * graph-mode calls are stream-ordered and return without waiting; the
 * persistent mode synchronises the stream to read the work queue's error
 * flag.  The streams mode runs hj_solve_brt of every instance (its own
 * kernel, launch configuration and solve graph; a first solve may autotune
 * and synchronise) on four private streams forked from the batch stream and
 * joined back into it, so the call is stream-ordered too; instances go to the
 * least-loaded stream in decreasing order of nodes x steps; tile settings do
 * not apply.  HJ_ERR_NOT_READY if an instance has no target; HJ_ERR_DEVICE
 * if a persistent tile waited past the spin limit (values then undefined). */
hj_status hj_batch_solve(hj_batch *b, const double *horizons, int32_t mode, hj_solve_info *infos);

/* Tile shape: x planes per tile for every instance (0 = the default: 16 for
 * streaming tiles, 32 for the batched plane kernel). */
hj_status hj_batch_set_tile(hj_batch *b, int32_t x_planes);

/* Polls a persistent tile makes of its dependency counter before it gives up
 * and raises the error flag (default 2^21, about a second; 0 = give up at
 * once).  The kernel always ends. */
hj_status hj_batch_set_spin_limit(hj_batch *b, int64_t polls);

/* Time complete batch solves (horizons, mode) for each candidate tile
 * length (4, 8, 12, 16, 24, 32, 48, 80 x planes), keep the fastest and
 * report it.  Synchronises; leaves every instance holding its solve.  The
 * streams mode has no tiles: HJ_ERR_INVALID_ARG. */
hj_status hj_batch_autotune(hj_batch *b, const double *horizons, int32_t mode, int32_t *x_planes_out);

hj_status hj_batch_get_info(hj_batch *b, hj_batch_info *out);

/* ---- Serving: continuous batching of re-solves ----------------------------
 * The paper's use is a robot re-solving its BRT whenever the obstacle map
 * changes (section "Hardware Correctness": V0 handed to the solver, the BRT
 * read back).  A server keeps grids resident on the device ("slots": the
 * handle's arrays, table and CFL step).  Each tick admits queued requests
 * (first in, first out) while fewer than max_inflight run and a slot is free
 * or the budget allows a new one, then advances running requests by a few
 * time steps.  Which ones, by `policy`:
 *   HJ_SERVE_SMALL_FIRST: requests of fewer than 4 Mi nodes (too small to
 *     fill the device alone) first, least remaining work (nodes times steps
 *     left) first, then the larger ones in the order they were submitted;
 *     requests are taken in that order until they hold 4 Mi nodes, the
 *     others wait for a later tick; requests older than age_ms (since
 *     submission) go first, oldest first, so past that age the order is
 *     first come, first served and no request waits without bound;
 *   HJ_SERVE_SHARE: every running request, every tick.
 * Among the requests of a tick, grids of fewer than 4 Mi nodes share one
 * launch per stage and step (each at its own step), larger ones fill the
 * device alone and step with their own stage kernel, and so does a small
 * one that is alone in its tick.  Every request
 * restarts from its own V0 and gets exactly the V of hj_solve_brt on a fresh
 * handle (bitwise), whatever the policy. */
enum { HJ_SERVE_SMALL_FIRST = 0, HJ_SERVE_SHARE = 1 };
typedef struct hj_server hj_server;

typedef struct {
  hj_scheme_desc scheme; /* one scheme for all requests */
  int64_t hbm_budget;    /* device bytes the slots may hold (0 = no limit); idle slots are freed to fit */
  int32_t max_inflight;  /* most requests stepping together (1..256) */
  int32_t x_planes;      /* tile length in x planes (0 = cut x so each launch has ~1024 blocks) */
  int32_t steps_per_tick; /* time steps one tick enqueues for the running requests (0 = 4); at most
                           * two ticks are in flight, so new requests wait for <= 2 ticks */
  int32_t policy;        /* HJ_SERVE_SMALL_FIRST or HJ_SERVE_SHARE */
  double age_ms;         /* small-first: age (ms since submission) after which a request goes first (0 = 5) */
} hj_server_desc;

typedef struct {
  int64_t submitted, admitted, completed, ticks;
  int32_t running, queued, slots, pad;
  int64_t slot_bytes; /* device bytes held by slots */
} hj_server_stats;

/* All work goes to hip_stream (borrowed; NULL = the null stream). */
hj_status hj_server_create(const hj_server_desc *desc, void *hip_stream, hj_server **out);
hj_status hj_server_destroy(hj_server *s);

/* Queue a re-solve of the BRT of the union of m cylinders (cx, cy, r:
 * centres and radii, copied) on `grid` with `dyn`, over `horizon`.  Nothing
 * runs until hj_server_tick.  HJ_ERR_OUT_OF_MEMORY if one slot of this grid
 * is larger than the whole budget. */
hj_status hj_server_submit(hj_server *s, const hj_grid_desc *grid, const hj_dynamics_desc *dyn, const double *cx,
                           const double *cy, const double *r, int32_t m, double horizon, int64_t *id);

/* Admit, then advance every running request by up to steps_per_tick time
 * steps (one launch per stage and step over the requests still short of
 * their horizon; stream-ordered, returns without waiting).  Requests that
 * arrive meanwhile join at the next tick.  *running = requests still
 * stepping. */
hj_status hj_server_tick(hj_server *s, int32_t *running);

/* Ids (up to cap) of requests whose V is complete on the device (event
 * queries; never waits). */
hj_status hj_server_poll(hj_server *s, int64_t *ids, int32_t cap, int32_t *n);

/* Copy a complete request's V (layout of hj_get_value; out may be NULL to
 * drop it) and give its slot back.  HJ_ERR_NOT_READY until poll lists it. */
hj_status hj_server_take(hj_server *s, int64_t id, void *out, int32_t dtype, int32_t where);

hj_status hj_server_get_stats(hj_server *s, hj_server_stats *out);

/* Message for the last failed call on this thread ("" if none). */
const char *hj_last_error(void);

/* Library version string. */
const char *hj_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HJ_H */
