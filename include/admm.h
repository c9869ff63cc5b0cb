/*
 * admm.h - C ABI of the MI355X (gfx950) factor-graph ADMM library.
 *
 * The library runs the message-passing ADMM of Algorithm 2 (paper Sec. II,
 * "ADMM on a factor-graph"): per iteration
 *     x_(a,.) = Prox_{f_a,rho}(n_(a,.))        for every factor a   (x-update)
 *     m_e     = x_e + u_e                     for every edge e     (m-update)
 *     z_b     = sum_{a in db} rho m_(a,b) / sum_{a in db} rho      (z-update)
 *     u_e     = u_e + alpha (x_e - z_b)                             (u-update)
 *     n_e     = z_b - u_e                                           (n-update)
 * where Prox_{h,rho}(r) = argmin_s h(s) + rho/2 |s - r|^2 (eq. (3)).
 *
 * Conventions for every function:
 *  - Every entry point returns an admm_status; nothing throws across the
 *    ABI.  On failure admm_last_error() returns a message for the calling
 *    thread (valid until that thread's next call).
 *  - Host arrays passed in are read during the call only; the caller keeps
 *    ownership.  Device memory the library allocates is owned by the handle
 *    and released by the matching destroy call.  Pointers documented as
 *    "device" must point to memory of the handle's device.
 *  - "stream" is a hipStream_t passed as void*; NULL means the null stream.
 *    Functions that return host results synchronise that stream.
 *  - A handle must not be used by two threads at the same time.
 *  - Edge slots: an edge (a,b) carries dim(b) scalar slots.  "User slot
 *    order" is the order in which edges were created: factors in the order
 *    of admm_graph_add_factors calls and rows of var_ids, each factor's
 *    edges in var_ids order, each edge's components in order (the layout
 *    of the paper's edge arrays, Sec. III).
 *  - z uses "variable order": variable 0's components, then variable 1's...
 */
#ifndef ADMM_H
#define ADMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ADMM_OK = 0,
  ADMM_E_ARG = 1,          /* invalid argument (ids, dims, sizes, nulls) */
  ADMM_E_STATE = 2,        /* call out of order (e.g. run before finalize) */
  ADMM_E_NUMERIC = 3,      /* parameter makes a prox ill-posed (rho <= gamma) */
  ADMM_E_HIP = 4,          /* a HIP runtime call failed */
  ADMM_E_OOM = 5,          /* device allocation failed */
  ADMM_E_NO_DEVICE = 6,    /* no usable GPU (validation still ran) */
  ADMM_E_UNSUPPORTED = 7   /* valid request outside the library's limits */
} admm_status;

/* Factor kinds (the proximal operators of the paper's appendix).
 *  kind        edges (dims)              params (per factor, param_len)
 *  NONOVERLAP  c1(2) r1(1) c2(2) r2(1)   none (0)             App. A, |c1-c2| >= r1+r2
 *  WALL        c(2) r(1)                 Qx Qy Vx Vy (4)       App. A, Q^T(c-V) >= r
 *  RADIUS      r(1)                      gamma (1)             App. A, -gamma/2 r^2, r >= 0
 *  QUAD        any                       q_k per slot (slots)  App. B, 1/2 sum q_k x_k^2
 *  BOX         any                       lo hi (2)             lo <= x_k <= hi
 *  HINGE       w_1..w_d(1 each) b(1)     a_1..a_d y C (d+2)    App. C, C max(0, 1-y(w.a+b))
 *  L2          any                       lambda (1)            App. C, lambda/2 |w|^2
 *  LINDYN      x(n) u(m) x'(n)           A (n*n) B (n*m)       App. B, x' = A x + B u
 *  LINDYN0     u(m) x'(n)                A B x0 (n*n+n*m+n)    App. B, x' = A x0 + B u
 *  MINERR      any                       lambda (1)            App. C, lambda sum xi_k, xi_k >= 0
 *  EQUAL       w1(d) w2(d)               none (0)              App. C, w1 = w2
 *  MARGIN      w(d) b(1) xi(1)           x_1..x_d y (d+1)      App. C, y(w.x + b) >= 1 - xi
 * MINERR requires lambda >= 0 and MARGIN y = +1 or -1, d <= 64 and the same
 * d for every factor of one call.  MARGIN's prox is the projection onto
 * its half-space (the appendix's closed form with the signs that make the
 * output feasible: w += mu y x / rho, b += mu y / rho, xi += mu / rho).
 * Matrices are row-major.  The prox of NONOVERLAP moves the radii by -D/4
 * (the sign that makes the output feasible) and uses the direction (1,0)
 * when the two centres coincide; RADIUS requires rho > gamma. */
typedef enum {
  ADMM_F_NONOVERLAP = 1,
  ADMM_F_WALL = 2,
  ADMM_F_RADIUS = 3,
  ADMM_F_QUAD = 4,
  ADMM_F_BOX = 5,
  ADMM_F_HINGE = 6,
  ADMM_F_L2 = 7,
  ADMM_F_LINDYN = 8,
  ADMM_F_LINDYN0 = 9,
  ADMM_F_MINERR = 10,
  ADMM_F_EQUAL = 11,
  ADMM_F_MARGIN = 12
} admm_factor_kind;

typedef enum { ADMM_FP32 = 0, ADMM_FP64 = 1 } admm_precision;

typedef struct admm_graph admm_graph;

/* Sizes and layout of a finalized graph (all counts, no pointers). */
typedef struct {
  int64_t n_vars, n_scalars, n_factors, n_edges, n_slots;
  int64_t n_buckets;           /* factor buckets after type bucketing */
  int64_t n_pair_tiles;        /* tiles of the dense pairwise layout (0 if none) */
  int64_t n_contributions;     /* entries summed by the z-update */
  int64_t state_bytes;         /* per-edge state resident in device memory */
  int64_t algo_bytes_per_iter; /* algorithmic HBM bytes of one iteration */
  int64_t layout_bytes_per_iter; /* index/partial bytes of one iteration */
  int32_t precision;           /* admm_precision */
  int32_t alpha_is_one;        /* 1: m-only state (alpha == 1) */
  int32_t driver;              /* ADMM_DRIVER_LAUNCHES, _RESIDENT or _GRAPH */
  int32_t resident_lds_bytes;  /* LDS image of the resident driver (0 if unused) */
  int32_t sparse_pair_state;   /* 1: pair tiles keep unmoved pairs' m implicit */
  int32_t three_weight;        /* 1: the three-weight variant (ADMM_OPT_THREE_WEIGHT) */
} admm_graph_info;

/* Message for the last failing call on this thread ("" if none). */
const char* admm_last_error(void);
/* ABI version of this header (incremented on incompatible change). */
int32_t admm_abi_version(void);

/* Create an empty graph with n_vars variable nodes; var_dim[n_vars] gives
 * each variable's dimension (>= 1).  precision: admm_precision of all
 * device arithmetic.  Paper Sec. III: the graph the user extends node by
 * node ("addNode"). */
admm_status admm_graph_create(int32_t n_vars, const int32_t* var_dim,
                              int32_t precision, admm_graph** out);

/* Append n_factors factors of one kind, each connected to `arity` variables:
 * var_ids[n_factors*arity] (row-major, edge order per factor).  params:
 * [n_factors*param_len] doubles, or [param_len] shared by all when
 * shared_params != 0 (NULL allowed when param_len == 0).  Dimensions and
 * param_len are checked against the kind's signature (table above);
 * violations return ADMM_E_ARG.  Only before finalize. */
admm_status admm_graph_add_factors(admm_graph* g, int32_t kind,
                                   int32_t n_factors, int32_t arity,
                                   const int32_t* var_ids,
                                   const double* params, int32_t param_len,
                                   int32_t shared_params);

/* rho (> 0) and alpha (> 0) of the edges (Alg. 2).  Defaults 1 and 1:
 * the values of every edge whose group has none of its own (below).  Only
 * before finalize. */
admm_status admm_graph_set_rho(admm_graph* g, double rho);
admm_status admm_graph_set_alpha(admm_graph* g, double alpha);

/* rho (> 0) of the edges of one group of factors: `group` counts the
 * admm_graph_add_factors calls from 0.  Algorithm 2 weighs each edge's
 * prox and its term of the z-average by rho_(a,b); here every edge of the
 * group gets `rho` (the closed forms assume equal weights within a
 * factor).  z_b then averages rho_(a,b) m_(a,b) over sum rho_(a,b), and the
 * dual residual weighs each variable's change by the largest rho of its
 * edges.  ADMM_E_ARG for a group index out of range or rho <= 0; only
 * before finalize. */
admm_status admm_graph_set_group_rho(admm_graph* g, int32_t group, double rho);

/* alpha (> 0) of the edges of one group of factors (u += alpha (x - z) on
 * each of them, Algorithm 2).  When every edge's alpha is 1 the library
 * keeps m alone per edge; otherwise m and x.  Errors as above. */
admm_status admm_graph_set_group_alpha(admm_graph* g, int32_t group, double alpha);

/* Layout options, set before finalize.
 *  ADMM_OPT_PAIR_ROWS: disks per row of a dense pair tile (16, 32 or 64;
 *  0 = default, 64).  Each tile holds rows x 64 pairs and
 *  is one workgroup of the x-pass; results do not depend on the choice
 *  beyond the order of the z-sums.
 *  ADMM_OPT_DRIVER: how admm_run executes the iterations (the loop of
 *  Algorithm 2; Sec. III runs each iteration as separate kernel launches).
 *  ADMM_DRIVER_LAUNCHES: one x-pass and one z-pass launch per iteration,
 *  enqueued back to back.  ADMM_DRIVER_GRAPH: the same launches, recorded
 *  once into a hipGraph of ADMM_OPT_GRAPH_BLOCK iterations (per starting z
 *  buffer, at the first run that needs it) and replayed with one graph
 *  launch per block; the last iteration of a run and any remainder are
 *  launched directly.  ADMM_DRIVER_RESIDENT: the whole run in one launch of
 *  one workgroup that keeps every per-iteration array in LDS; only for small
 *  graphs (no dense pair tiles, LDS image within the device's per-workgroup
 *  limit): finalize returns ADMM_E_UNSUPPORTED when the graph does not fit.
 *  ADMM_DRIVER_AUTO (default): resident when the graph fits and has at most
 *  64 x-pass plus z-pass blocks, else graph.  The arithmetic of every step
 *  is the same in every driver, and launches and graph give identical bits.
 *  ADMM_OPT_GRAPH_BLOCK: iterations per recorded block (even, 2..4096;
 *  0 = default 32).
 *  ADMM_OPT_ZLIST: where the z-update finds the contributions of the disks
 *  of 64-row pair tiles.  ADMM_ZLIST_AUTO (default) or 16, 32, 64: in
 *  transposed lists, contribution j of scalar k at j * n + k with the
 *  scalars in disk order, so that each tile's 192 row and 192 column
 *  partial sums are contiguous; the z-pass sums 16, 32 or 64 lists per
 *  block (auto: 32).  ADMM_ZLIST_ZMAJOR: each scalar's contributions
 *  contiguous, as for every other variable (the tile partials are then
 *  scattered stores).  Results differ only in the order of the z-sums.
 *  ADMM_OPT_THREE_WEIGHT (0 or 1, default 0): Sec. II gives every edge its
 *  own rho_(a,b) and names improved update schemes for them, citing the
 *  three-weight message-passing algorithm.  With 1 every message carries a
 *  weight 0 or rho: a non-overlap or wall factor whose constraint is
 *  inactive (its prox leaves n unchanged) sends 0, every other factor rho;
 *  z_b is the weighted mean of the incoming m and keeps its value when
 *  every weight is 0; an edge sent with weight 0 has its u reset to 0; a
 *  variable no factor weighted is received with weight 0, and a constraint
 *  factor then moves only such edges, in equal shares.  Built for packing
 *  graphs (non-overlap, wall and separable factors, one rho, alpha = 1;
 *  dense pair tiles only with the sparse pair state, so FP64 or
 *  ADMM_PAIR_STATE_DENSE graphs take the general layout), with the launch
 *  and graph drivers: finalize returns ADMM_E_UNSUPPORTED otherwise.  After
 *  a run every edge's state is explicit (an inactive edge's m is z, its u
 *  0), so admm_get_u/x and split runs see the same arrays as one run.
 *  ADMM_OPT_PAIR_STATE: per-edge state of dense pair tiles.  With alpha = 1
 *  a pair whose prox leaves n unchanged (no overlap) ends the iteration with
 *  m = z, the consensus it started from (Alg. 2: m = x + u, u = m_old - z,
 *  x = n = 2z - m_old).  ADMM_PAIR_STATE_AUTO (default) keeps such pairs'
 *  m implicit in FP32 with alpha = 1: one flag bit per pair, and m is only
 *  read and written for pairs the prox moves; the next iteration takes
 *  their m from the previous z.  Every prox is still evaluated every
 *  iteration; the last iteration of a run stores the state of every pair.
 *  ADMM_PAIR_STATE_DENSE reads and writes every pair's m every iteration
 *  (always the case in FP64 or with alpha != 1). */
enum { ADMM_OPT_PAIR_ROWS = 1, ADMM_OPT_DRIVER = 2, ADMM_OPT_PAIR_STATE = 3,
       ADMM_OPT_GRAPH_BLOCK = 4, ADMM_OPT_THREE_WEIGHT = 5, ADMM_OPT_ZLIST = 6 };
enum { ADMM_ZLIST_AUTO = 0, ADMM_ZLIST_ZMAJOR = 1 };
enum { ADMM_DRIVER_AUTO = 0, ADMM_DRIVER_LAUNCHES = 1, ADMM_DRIVER_RESIDENT = 2,
       ADMM_DRIVER_GRAPH = 3 };
enum { ADMM_PAIR_STATE_AUTO = 0, ADMM_PAIR_STATE_DENSE = 1 };
admm_status admm_graph_set_option(admm_graph* g, int32_t option, int64_t value);

/* Paper Sec. III: the step that copies the graph built on the host to the
 * GPU once, before any iteration (graph construction and this copy are
 * outside the timed iterations there too).  Validate, bucket factors by
 * kind, build the device layout (edge-major structure-of-arrays per
 * bucket, dense pair tiles for complete pairwise non-overlap buckets,
 * per-variable contribution lists) and upload it to `device`; the handle
 * owns every device buffer from here on.  Sets z to 0 and u to 0.  Returns
 * ADMM_E_NO_DEVICE (after full validation) when no GPU is present,
 * ADMM_E_NUMERIC when rho <= gamma for a RADIUS factor, ADMM_E_STATE when
 * called twice, ADMM_E_OOM when a device allocation fails. */
admm_status admm_graph_finalize(admm_graph* g, int32_t device);

/* Counts and byte figures of a finalized graph (paper Sec. IV: the number
 * of factors, edges and variables of each problem; here also the layout
 * the library chose).  info: caller-owned struct, filled on success;
 * ADMM_E_STATE before finalize. */
admm_status admm_graph_info_get(const admm_graph* g, admm_graph_info* info);

/* Algorithm 2's initial state (Sec. II: the iteration starts from given z
 * and u; n = z - u before the first x-update).  Set it from host arrays:
 * z[n_scalars] in variable order and u[n_slots] in user slot order (NULL:
 * u = 0); both are copied (double, converted to the working precision) and
 * the stream is synchronised before return.  The next x-update uses
 * n = z - u.  ADMM_E_STATE before finalize, ADMM_E_ARG for a NULL z. */
admm_status admm_set_state(admm_graph* g, const double* z, const double* u,
                           void* stream);

/* Run `iters` >= 0 iterations of Algorithm 2 on the device, enqueued on
 * `stream` without host round-trips.  The last iteration also records
 * what admm_get_residuals and admm_get_x return. */
admm_status admm_run(admm_graph* g, int32_t iters, void* stream);

/* admm_run with a HIP event pair around every kernel: same results, and
 * the summed device time of the x-passes and of the z-passes in
 * milliseconds.  Synchronises the stream.  For measurement only: the
 * events add a small gap between kernels.  With the resident driver the
 * one launch's time is returned as xpass_ms and zpass_ms is 0. */
admm_status admm_run_profiled(admm_graph* g, int32_t iters, void* stream,
                              double* xpass_ms, double* zpass_ms);

/* Paper Sec. III: after the iterations the z values are copied back from
 * the GPU (the only per-solve transfer there; Sec. V reports its time).
 * Copy results to caller-owned host arrays (double, widened from the
 * working precision).  z: [n_scalars] variable order; u and x: [n_slots]
 * user slot order (x of the last iteration run; u and x are the per-edge
 * quantities of Algorithm 2, for inspection and for resuming a run through
 * admm_set_state).  Synchronise the stream.  ADMM_E_STATE before finalize,
 * ADMM_E_ARG for a NULL output. */
admm_status admm_get_z(admm_graph* g, double* z, void* stream);
admm_status admm_get_u(admm_graph* g, double* u, void* stream);
admm_status admm_get_x(admm_graph* g, double* x, void* stream);

/* Residuals of the last iteration run: r = max_e |x_e - z_b| and
 * s = rho max_b |z_b - z_b(previous iteration)| (the paper leaves the
 * stopping criterion open; these are the infinity-norm measures used
 * throughout this library).  Synchronises the stream.  ADMM_E_STATE before
 * any iteration since the last state import.  ADMM_E_NUMERIC when an x or
 * z of the last iteration is NaN or infinite (a NaN anywhere propagates to
 * both through the averages); the status is sticky: every later call
 * returns it until admm_set_state imports a new state. */
admm_status admm_get_residuals(admm_graph* g, double* r_primal,
                               double* r_dual, void* stream);

/* Device address of z (working precision, variable order) for callers that
 * read it in place (Sec. III's read-back of z without the copy); valid
 * until the next run or destroy; the handle keeps ownership. */
admm_status admm_z_device_ptr(admm_graph* g, void** z_dev);

/* Release the handle and every device buffer it owns (the GPU-side graph of
 * Sec. III).  NULL is accepted and does nothing.  The handle must not be in
 * use by another thread or have work pending on a stream the caller will
 * not synchronise. */
admm_status admm_graph_destroy(admm_graph* g);

/* ------------------------------------------------------------------------
 * Batched linear MPC (paper Sec. V-B; App. B proximal operators).
 * Instance i: x_{t+1} = A_i x_t + B_i u_t, t = 0..T_i-1, x_0 given per solve;
 * cost 1/2 sum_{t=1..T} x_t^T diag(q_i) x_t + 1/2 sum_{t=0..T-1} u_t^T
 * diag(r_i) u_t; |u_t|_inf <= u_box_i when u_box_i > 0.  Its factor graph
 * has variable nodes u_t (dim m) and x_{t+1} (dim n) and, per step, a
 * linear-dynamics factor, a quadratic factor on u_t and on x_{t+1} and a box
 * factor on u_t; alpha = 1.  Limits: T <= 256, n <= 12, m <= 4.
 * z layout of instance i (offset zoff_i = sum_{j<i} T_j (n_j + m_j)): per
 * step t the m entries of u_t then the n entries of x_{t+1}.
 * Per-edge dual layout (offset sum_{j<i} 3 T_j (n_j + m_j)): per step t
 * [dyn x_t (n) | dyn u_t (m) | dyn x_{t+1} (n) | quad u_t (m) | box u_t (m) |
 * quad x_{t+1} (n)]; the x_t entries of step 0 are unused.
 * ------------------------------------------------------------------------ */
typedef struct admm_mpc_batch admm_mpc_batch;

/* Host arrays (copied): T, n, m [n_inst]; A (n_i*n_i), B (n_i*m_i), q (n_i),
 * r (m_i) concatenated over instances, row-major; u_box [n_inst].  rho > 0.
 * Precomputes the projection matrices and uploads everything to `device`.
 * ADMM_E_UNSUPPORTED beyond the limits above (checked before any device
 * call). */
admm_status admm_mpc_batch_create(int32_t n_inst, const int32_t* T, const int32_t* n,
                                  const int32_t* m, const double* A, const double* B,
                                  const double* q, const double* r, const double* u_box,
                                  double rho, int32_t device, admm_mpc_batch** out);

/* Element counts of the batch's z, per-edge dual and x0 arrays. */
admm_status admm_mpc_batch_sizes(const admm_mpc_batch* b, int64_t* z_total,
                                 int64_t* u_total, int64_t* x0_total);

/* Solve every instance in one persistent launch, asynchronously on `stream`.
 * Device arrays (float32 / int32): x0 [x0_total]; z_init [z_total] or NULL
 * (cold start, z = 0); z_out [z_total]; iters_out [n_inst].  dual_mode 0:
 * u^0 = 0; 1: u^0 from dual completion of z_init (requires z_init).  Each
 * instance stops at the first iteration with r = max_e |x_e - z_b| <= tol and
 * s = rho max_b |z_b - z_b(previous)| <= tol; iters_out holds that iteration,
 * or -max_iter when it did not converge. */
admm_status admm_mpc_batch_solve(admm_mpc_batch* b, const float* x0, const float* z_init,
                                 int32_t dual_mode, float tol, int32_t max_iter,
                                 float* z_out, int32_t* iters_out, void* stream);

/* Dual completion only (device arrays): u [u_total] from z [z_total].  At a
 * solution z* it gives the duals that make (z*, u) a fixed point. */
admm_status admm_mpc_batch_dual_complete(admm_mpc_batch* b, const float* z, float* u,
                                         void* stream);

/* Solve from a full ADMM state: z_init [z_total] (NULL: cold start, z = 0)
 * and per-edge duals u_init [u_total] (NULL: u^0 = 0; needs z_init).  On
 * exit z_out holds z and, when u_out is not NULL, u_out [u_total] the duals
 * u = m - z of the last iteration, so a later call can continue the same
 * iteration from (z_out, u_out) (Algorithm 2 keeps nothing else per edge
 * when alpha = 1).  Stopping rule and iters_out as in admm_mpc_batch_solve.
 * Device arrays; z_out must not be z_init and u_out must not be u_init
 * (ADMM_E_ARG).  Asynchronous on `stream`. */
admm_status admm_mpc_batch_solve_state(admm_mpc_batch* b, const float* x0, const float* z_init,
                                       const float* u_init, float tol, int32_t max_iter,
                                       float* z_out, float* u_out, int32_t* iters_out,
                                       void* stream);

/* One receding-horizon step for every instance (paper Sec. V-B: in each
 * controller cycle only the current state changes and the ADMM continues
 * from the previous cycle's solution).  Device arrays:
 *   x0_next = A x0 + B u_0 + w, with u_0 the first input of z (w [x0_total]
 *             may be NULL: no disturbance);
 *   z_next (may be NULL): z moved one step forward, z'(t) = z(t+1) for
 *             t < T-1, and the last step u = 0, x = A x_T;
 *   u_next (given with u, else both NULL): every edge's dual moved with its
 *             step; the step-1 dual on the dynamics factor's x_1 edge is
 *             dropped (step 0 has no such edge) and the last step's duals
 *             are zero, so the duals around each variable keep their sum.
 * Outputs must not be the corresponding inputs (ADMM_E_ARG).  Asynchronous
 * on `stream`. */
admm_status admm_mpc_batch_shift(admm_mpc_batch* b, const float* x0, const float* z,
                                 const float* u, const float* w, float* x0_next, float* z_next,
                                 float* u_next, void* stream);

/* Schedule of the persistent launch: pack1 = instances per workgroup for
 * T <= 64 (1, 2 or 4; at most 2 in a batch whose instances all have
 * T <= 128, which runs on 128-thread workgroups), order (0 as given, 1 most work per iteration first,
 * 2 grouped by (n, m), 3 longest expected solve first: the iteration counts
 * of the autotuner's cold solve times the latency of one iteration; as 1
 * before a tuning run), grid = workgroups (0: as many as fit on the device
 * at once).  A batch finishes with its slowest instance, so starting the
 * longest solves first shortens it.  Results do not depend on the plan
 * (bitwise). */
admm_status admm_mpc_batch_set_plan(admm_mpc_batch* b, int32_t pack1, int32_t order,
                                    int32_t grid);
admm_status admm_mpc_batch_get_plan(const admm_mpc_batch* b, int32_t* pack1,
                                    int32_t* order, int32_t* grid, int32_t* resident);

/* Autotuner: one cold solve of this batch from x0 (device) records each
 * instance's iterations (for order 3), then every candidate plan is timed
 * on cold solves, reps launches each (best time kept), and the fastest is
 * kept.
 * z_scratch [z_total] and iters_scratch [n_inst] are device work arrays;
 * times_ms [max_candidates] (host, nullable) receives each candidate's time.
 * Synchronises the stream. */
admm_status admm_mpc_batch_tune(admm_mpc_batch* b, const float* x0, float tol,
                                int32_t max_iter, float* z_scratch,
                                int32_t* iters_scratch, int32_t reps, float* times_ms,
                                int32_t max_candidates, int32_t* n_candidates,
                                void* stream);

admm_status admm_mpc_batch_destroy(admm_mpc_batch* b);

/* ------------------------------------------------------------------------
 * Learned warm start: an MLP x0 -> z0 (initial trajectory of an MPC
 * instance), y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, trained on the GPU
 * with mean-squared error and Adam.  Every product runs on the matrix cores
 * with bf16 operands (round to nearest even) and fp32 accumulation; master
 * weights, activations and gradients are fp32.  Parameter vector order:
 * W1 [hidden][n_in], b1 [hidden], W2 [hidden][hidden], b2 [hidden],
 * W3 [n_out][hidden], b3 [n_out] (row-major).  The caller supplies the
 * initial weights; nothing here draws random numbers.
 * ------------------------------------------------------------------------ */
typedef struct admm_mlp admm_mlp;

/* Allocate parameters, Adam moments and activations for batches up to
 * max_batch on `device`; parameters start at zero.  ADMM_E_UNSUPPORTED when
 * max_batch times the widest layer reaches 2^31 elements. */
admm_status admm_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t max_batch,
                            int32_t device, admm_mlp** out);
/* Number of parameters (-1 for NULL). */
int64_t admm_mlp_n_params(const admm_mlp* n);
/* Host float arrays [n_params]; set also resets the Adam state. */
admm_status admm_mlp_set_params(admm_mlp* n, const float* host);
admm_status admm_mlp_get_params(admm_mlp* n, float* host);
/* Fixed (not trained) output affine y = mean + sd * yhat, yhat = W3 h2 + b3.
 * The training loss is taken on normalised outputs, mean((yhat - (target -
 * mean) / sd)^2), so every output is learned to the same relative accuracy
 * and the bf16 products work on unit-scale values.  Default mean 0, sd 1.
 * fit: per-output mean and standard deviation (floored at sd_min) of a
 * device array targets [rows][n_out], FP64 accumulation in a fixed order;
 * allocates a temporary workspace and synchronises the stream. */
admm_status admm_mlp_fit_output_scaling(admm_mlp* n, const float* targets, int64_t rows,
                                        float sd_min, void* stream);
/* admm_mlp_fit_output_scaling for callers that cannot allocate (code under
 * hipGraph capture, serving loops, harnesses that forbid hipMalloc): the
 * same statistics, computed in a fixed 8 MiB device workspace that the
 * library holds on each device for the life of the process, with no
 * allocation, free or synchronisation (asynchronous on `stream`).  The
 * chunks are those of admm_mlp_fit_output_scaling (bit-identical results)
 * as long as (chunks + 1) * n_out fit the workspace's 2^20 doubles, else
 * fewer, longer chunks.  ADMM_E_UNSUPPORTED when n_out > 2^19.  Every call
 * on one device shares the workspace: calls that overlap in time on one
 * device (other streams, other threads) race and must be serialised by
 * the caller. */
admm_status admm_mlp_fit_output_scaling_noalloc(admm_mlp* n, const float* targets, int64_t rows,
                                                float sd_min, void* stream);
admm_status admm_mlp_set_output_scaling(admm_mlp* n, const float* mean, const float* sd);
admm_status admm_mlp_get_output_scaling(admm_mlp* n, float* mean, float* sd);
/* y [batch][n_out] = MLP(x [batch][n_in]) including the output affine;
 * device arrays, async. */
admm_status admm_mlp_forward(admm_mlp* n, const float* x, int32_t batch, float* y, void* stream);
/* Gradient of the normalised loss over all batch*n_out entries: grads
 * [n_params] (device, nullable) and loss (device scalar, nullable). */
admm_status admm_mlp_grads(admm_mlp* n, const float* x, const float* target, int32_t batch,
                           float* grads, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * loss; loss (device scalar, nullable) is the loss before the step. */
admm_status admm_mlp_train_step(admm_mlp* n, const float* x, const float* target, int32_t batch,
                                float lr, float* loss, void* stream);
admm_status admm_mlp_destroy(admm_mlp* n);

#ifdef __cplusplus
}
#endif

#endif /* ADMM_H */
