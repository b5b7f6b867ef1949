/*
 * amg.h -- C ABI of the MI355X (gfx950) solver for graph-Laplacian systems
 *
 *     (Au, v) = sum_{e=(i,j) in E} w_e (u_i - u_j)(v_i - v_j) + sum_{i in S_b} d_i u_i v_i = (f, v)
 *
 * (eq. (prob), Section 1 of Brannick, "Aggregation-based aggressive coarsening
 * with polynomial smoothing"), solved by flexible CG preconditioned by a
 * nonlinear AMLI cycle (k-cycle) over unsmoothed-aggregation coarse levels with
 * the polynomial smoother of best uniform approximation to 1/x (Sections 3-4).
 *
 * Conventions shared by every call:
 *   - All integers are int32 unless stated; all floating point is IEEE binary64
 *     at the boundary.
 *   - "host pointer": ordinary CPU memory, read during the call only; the
 *     library copies what it keeps.  "device pointer": memory on the current
 *     HIP device (e.g. a torch tensor's data_ptr()), never freed by the library.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     ordered on that stream; calls that return results to the host synchronize
 *     it.
 *   - Every call returns AMG_OK (0) or a negative amg_status.  Argument and graph
 *     validation happens on the host before any device call, so invalid input is
 *     reported identically with or without a GPU.
 *   - A hierarchy handle owns all device memory it allocated until amg_free.
 *     Calls on one handle must not overlap in time (they share its workspace).
 */
#ifndef AMG_H
#define AMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMG_OK = 0,
  AMG_ERR_ARG = -1,          /* null pointer, bad size or bad parameter value      */
  AMG_ERR_GRAPH = -2,        /* malformed CSR: range, order, self loop, asymmetry,
                                w <= 0 or non-finite, d < 0 or non-finite          */
  AMG_ERR_DISCONNECTED = -3, /* the graph is not connected                         */
  AMG_ERR_SINGULAR = -4,     /* all d_i = 0 (A singular) or a non-positive pivot
                                in the coarsest Cholesky factorization             */
  AMG_ERR_DEGREE = -5,       /* smoother error E_m >= 1 for the requested degree   */
  AMG_ERR_COARSEN = -6,      /* coarsening stagnated above max_coarsest rows       */
  AMG_ERR_NOMEM = -7,        /* device allocation failed                           */
  AMG_ERR_DEVICE = -8,       /* no usable HIP device, or a HIP runtime error       */
  AMG_ERR_BREAKDOWN = -9,    /* outer FCG: (p, Ap) <= 0 or non-finite              */
  AMG_ERR_MAXIT = -10,       /* max_iter reached before tol (u is still written)   */
  AMG_ERR_BUDGET = -11       /* request does not fit the HBM budget                */
} amg_status;

enum { AMG_FP64 = 0, AMG_MIXED = 1 };
enum { AMG_KEY_NORMALIZED = 0, AMG_KEY_RAW = 1 };
enum { AMG_TIE_INDEX = 0, AMG_TIE_HASH = 1 };
enum { AMG_CYCLE_K = 0, AMG_CYCLE_AMLI = 1 };
enum { AMG_AGG_MATCHING = 0, AMG_AGG_MIS = 1 };
enum { AMG_STOP_RESIDUAL = 0, AMG_STOP_ENERGY = 1 };

#define AMG_MAX_LEVELS 32

/*
 * Solver parameters (plain struct, passed by pointer, copied by amg_setup).
 *   degree        m of the smoother q_m (Section 3; Section 4 uses 4).  Must give
 *                 E_m = delta^m (kappa-1)/2 < 1, else AMG_ERR_DEGREE.  -1: the
 *                 smallest m with E_m <= smoother_rho and E_m < 1 (the bound on
 *                 m of Section 3, read with the consistent units of E_m < 1).
 *   smoother_rho  damping factor rho for degree = -1, in (0, 1] (default 0.33:
 *                 m = 4 at lambda0_ratio 10, the choice of Section 4).
 *   agg_size      target aggregate size; log2(agg_size) rounded = number of
 *                 matching passes per level (4 -> 2 passes, 16 -> 4).
 *   coarse_max    stop coarsening once a level has at most this many rows.
 *   lambda0_ratio lambda1 / lambda0 of the smoothing interval (Section 4: 10).
 *   inner_steps   flexible-CG steps per coarse level in the k-cycle (W-cycle: 2).
 *   restart       outer FCG keeps at most this many directions (Section 4: 5).
 *   tol           the stopping test's reduction factor (see stop).
 *   max_iter      outer iteration cap.
 *   precision     AMG_FP64, or AMG_MIXED: cycle, smoother and coarse-level
 *                 vectors and matrices in FP32 with FP32 accumulation; outer FCG,
 *                 every inner product, the coarsest factor and solve in FP64.
 *   match_key     AMG_KEY_NORMALIZED: edge strength W_ij^2/(D_i D_j);
 *                 AMG_KEY_RAW: W_ij.  Ties broken by the vertex indices (i, j).
 *   max_coarsest  largest coarsest level accepted when coarsening stagnates.
 *   stagnation    a level that keeps more than this fraction of its rows stops
 *                 the coarsening.
 *   use_graph     1: replay the cycle and the outer iteration as HIP graphs.
 *   tail_rows     the inner solve of the finest level with at most this many
 *                 rows whose data (with all coarser levels) fits in one
 *                 workgroup's LDS runs as one workgroup-resident kernel
 *                 (0 disables).
 *   autotune      1: choose every level's sliced-ELL layout at setup -- levels
 *                 of at least 262144 rows by timing the Chebyshev step on each
 *                 candidate layout, smaller ones by the bytes a pass moves;
 *                 0: use slice_height / lanes_per_row / sort_rows everywhere.
 *                 The layout never changes results: row sums are added in a
 *                 fixed order of classes and inner products in row order.
 *   slice_height  rows per slice: 8, 16, 32 or 64 (autotune = 0).
 *   lanes_per_row lanes that share one row's entries: 1, 2 or 4 (autotune = 0).
 *   sort_rows     1: rows ordered by decreasing length inside each group of 64
 *                 rows, which cuts padding on uneven degrees (autotune = 0).
 *   tie_break     order of edges of equal strength in the matching:
 *                 AMG_TIE_INDEX: by the vertex indices (i, j) (default);
 *                 AMG_TIE_HASH: by h(i, j), then (i, j), where h is MurmurHash3's
 *                 32-bit finalizer of (i * 2654435761 + j) mod 2^32 -- on
 *                 structured meshes this breaks the long index chains, so the
 *                 handshake needs far fewer rounds (a different hierarchy).
 *   cycle         AMG_CYCLE_K (default): the nonlinear AMLI cycle (k-cycle) of
 *                 Section 4 inside flexible CG; AMG_CYCLE_AMLI: the stationary
 *                 AMLI W-cycle, whose coarse correction is the degree-1 best
 *                 uniform approximation to 1/t on [a, 1] applied to the
 *                 preconditioned coarse operator (a estimated at setup by 20
 *                 power iterations on I - B A per level); needs inner_steps = 2.
 *                 The items of one batch share the cycle.
 *   aggregation   AMG_AGG_MATCHING (default): agg_size = 2^P from P heavy-edge
 *                 matching passes; AMG_AGG_MIS: Section 2's partitioning as the
 *                 paper's experiments use it -- a maximal independent set of
 *                 the graph of A^k (k = mis_distance; vertices taken in
 *                 decreasing splitmix64(index) priority), then every vertex
 *                 joins its nearest set vertex (ties: the smallest index).
 *   mis_distance  k of AMG_AGG_MIS, 1..8 (Section 4: 4).
 *   neumann       1: allow d = 0 everywhere (pure Neumann problem, A singular
 *                 with the constants as kernel): the coarsest factor is that of
 *                 A_L + (1/n_L) 1 1^T, a pseudo-inverse on right-hand sides
 *                 orthogonal to 1; the caller passes f orthogonal to 1.
 *   stop          AMG_STOP_RESIDUAL (default): ||r_k||_2 <= tol ||r_0||_2 on the
 *                 recursively updated residual.  AMG_STOP_ENERGY: Section 4's
 *                 test, the A-norm of the error reduced by tol, for the
 *                 homogeneous problem A u = 0 from the caller's initial guess
 *                 (f must be zero: amg_solve returns AMG_ERR_ARG otherwise);
 *                 the error is then the iterate itself, and (u_k, A u_k) is
 *                 formed from a fresh product each iteration (one extra
 *                 finest-level product).  On a pure Neumann problem
 *                 constants have A-norm 0.  Single solves only (the batched
 *                 and served forms reject it).
 *   fuse          1 (default): on levels below 2^18 rows, fold the inner
 *                 flexible-CG vector updates into the kernels that read them
 *                 and form the restriction of the residual in one pass; 0: one
 *                 launch per step.  Both give the same bits.
 */
typedef struct {
  int32_t degree;
  int32_t agg_size;
  int32_t coarse_max;
  double lambda0_ratio;
  int32_t inner_steps;
  int32_t restart;
  double tol;
  int32_t max_iter;
  int32_t precision;
  int32_t match_key;
  int32_t max_coarsest;
  double stagnation;
  int32_t use_graph;
  int32_t tail_rows;
  int32_t autotune;
  int32_t slice_height;
  int32_t lanes_per_row;
  int32_t sort_rows;
  int32_t tie_break;
  int32_t fuse;
  double smoother_rho;
  int32_t cycle;
  int32_t aggregation;
  int32_t mis_distance;
  int32_t neumann;
  int32_t stop;
} amg_params;

typedef struct amg_hier amg_hier;

/* Per-solve report.  rel_res is the ratio the stopping test uses (recursively
 * updated residual norms, or A-norms of the error under AMG_STOP_ENERGY);
 * rel_res_true = ||f - A u||_2 / ||f - A u0||_2 recomputed in FP64 at the end.
 * Under AMG_STOP_RESIDUAL a pass of the recursive test is confirmed on the
 * true FP64 residual, which then replaces the recursive one: AMG_OK means
 * rel_res_true <= tol; if it is above tol the outer iteration restarts from
 * it (counted in `replacements`) and goes on.
 * iters counts the outer iterations applied to u; test_iter is the iteration
 * whose stopping test passed (iters - 1 when the single solve had already
 * queued the next iteration before reading the test; = iters otherwise). */
typedef struct {
  int32_t status;
  int32_t iters;
  double rel_res;
  double rel_res_true;
  double solve_ms;
  int32_t test_iter;
  int32_t replacements;
} amg_info;

/* Hierarchy description (sizes, complexities and setup timings). */
typedef struct {
  int32_t levels;                     /* number of levels, finest = 0           */
  int32_t n[AMG_MAX_LEVELS];          /* rows per level                         */
  int64_t nnz[AMG_MAX_LEVELS];        /* stored off-diagonal entries per level  */
  double lambda1[AMG_MAX_LEVELS];     /* ||A_l||_inf per level                  */
  double grid_complexity;             /* sum n_l / n_0 (Section 4)              */
  double operator_complexity;         /* sum (nnz_l + n_l) / (nnz_0 + n_0)      */
  double setup_ms;                    /* whole amg_setup, device time           */
  double aggregation_ms;              /* matching passes (or independent set and
                                         nearest owners) + coarse numbering     */
  double galerkin_ms;                 /* coarse operators (sort and reduce)     */
  int32_t match_rounds;               /* handshake rounds summed over passes (or
                                         independent-set rounds over levels)    */
  int32_t precision;
  double device_bytes;                /* device memory held by the hierarchy    */
  double layout_ms;                   /* sliced-ELL layouts incl. autotuning    */
  int32_t slice_height[AMG_MAX_LEVELS];  /* chosen layout per smoothed level     */
  int32_t lanes_per_row[AMG_MAX_LEVELS];
  int32_t sorted_rows[AMG_MAX_LEVELS];
  int64_t sell_entries[AMG_MAX_LEVELS];  /* stored entries including padding    */
  int32_t degree;                     /* smoother degree in use                 */
  double amli_lambda_min[AMG_MAX_LEVELS];  /* AMLI: estimated lambda_min(B_l A_l), 0 elsewhere */
} amg_hier_desc;

/* Fill *p with the defaults: degree 4, agg_size 4, coarse_max 64,
 * lambda0_ratio 10, inner_steps 2, restart 5, tol 1e-8, max_iter 200, FP64,
 * normalized key, max_coarsest 2048, stagnation 0.9, use_graph 1,
 * tail_rows 4096, autotune 1 (fixed layout: slice_height 64, lanes_per_row 1,
 * sort_rows 0), index tie-breaking. */
void amg_params_default(amg_params* p);

/* Human-readable name of a status code (static string). */
const char* amg_strerror(int32_t status);

/* Detail message of the last failing call on this thread (static storage,
 * valid until the next failing call). */
const char* amg_last_error(void);

/*
 * Build the hierarchy for the graph of eq. (prob) (Sections 2-4): matching
 * aggregation passes, Galerkin coarse operators (the quotient graph of
 * Section 2 with summed weights), smoother intervals and coefficients, and the
 * Cholesky factor of the coarsest matrix, all computed on the device.
 *   n        number of vertices (>= 1)
 *   row_ptr  host, n+1 entries, row_ptr[0] = 0, non-decreasing
 *   col      host, row_ptr[n] entries: neighbours of each vertex, both
 *            directions stored, strictly increasing within a row, no self loop
 *   w        host, edge weights aligned with col; w_ij == w_ji > 0 exactly
 *   d        host, n lower-order terms d_i >= 0 (zero off S_b), not all zero
 *   params   host, NULL = defaults
 *   out      receives the handle (set to NULL on failure)
 * Errors: ARG, GRAPH, DISCONNECTED, SINGULAR, DEGREE (host validation, before
 * any device call); DEVICE, NOMEM, COARSEN, SINGULAR (device phase).
 */
int32_t amg_setup(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                  const double* d, const amg_params* params, void* stream, amg_hier** out);

/* Release every device allocation of the handle (NULL is accepted). */
void amg_free(amg_hier* h);

/* Describe the hierarchy (host struct). */
int32_t amg_describe(const amg_hier* h, amg_hier_desc* out);

/*
 * Solve A u = f by flexible CG preconditioned by the k-cycle (Section 4).
 *   f     device, n doubles
 *   u     device, n doubles: initial guess on entry, solution on exit
 *   info  host, may be NULL
 * Returns OK, MAXIT (u holds the last iterate), BREAKDOWN or DEVICE.  One
 * host synchronization per outer iteration (the stopping test).
 */
int32_t amg_solve(amg_hier* h, const double* f, double* u, void* stream, amg_info* info);

/*
 * amg_solve without allocating: for callers that cannot allocate device
 * memory or create runtime objects while they solve (code inside a tight
 * serving loop, harnesses that forbid allocation, work recorded around HIP
 * graph capture).  The same solve as amg_solve -- same kernels, same
 * arithmetic, same stopping test, same arguments and results -- except that
 *   - the reduction scratch (scalar area, arrival counter and block partials
 *     of the inner products) is a static device array of 4 MiB that each GPU
 *     holds from its first use until the process ends, instead of the
 *     hierarchy's own buffers;
 *   - no HIP graph, event or stream is created: outer iterations are launched
 *     directly and the host waits on the stream once per iteration (no
 *     iteration is queued ahead of the stopping test, so `iters` can be one
 *     lower than amg_solve's).
 * No hipMalloc, hipFree or other allocating call is made; the hierarchy's
 * workspace (allocated by amg_setup) holds the vectors.  Limit: the finest
 * level may have at most 16,739,328 rows (65,388 blocks of 256 rows of
 * partials); larger hierarchies return AMG_ERR_ARG with the limit in
 * amg_last_error().  The hierarchy must live on the current device
 * (AMG_ERR_ARG otherwise).  Every no-allocation solve on one GPU shares that
 * GPU's array and leaves its last contents there (the counter is cleared by
 * a fill kernel at the start of each call): two such solves that overlap in
 * time on one GPU (different streams or threads) race and give wrong
 * results; serialize them.
 */
int32_t amg_solve_noalloc(amg_hier* h, const double* f, double* u, void* stream, amg_info* info);

/* Duration of the finest level's interior Chebyshev step (one fused pass over
 * the level: w_{k+1} = 2 (A w_k - theta w_k)/eta - w_{k-1}, y += c_{k+1} w_{k+1};
 * the smoother of Section 3), the solve's dominant kernel.  amg_time_step
 * launches that kernel `reps` times back to back on `stream`, on the
 * hierarchy's own workspace (it overwrites the finest level's smoother
 * buffers, not the caller's vectors), between two HIP events, and reports the
 * mean time per launch.  Needs at least two levels. */
typedef struct {
  int32_t launches;     /* timed launches                           */
  double avg_ms;        /* event-to-event time / launches           */
  int32_t rows;         /* rows of the finest level                 */
  int64_t nnz;          /* stored off-diagonal entries              */
  int64_t entries;      /* sliced-ELL entries including padding     */
  int32_t grid;         /* workgroups per launch (256 rows each)    */
  int32_t value_bytes;  /* 8 (FP64 cycle) or 4 (mixed: FP32 cycle)  */
} amg_kernel_timing;

int32_t amg_time_step(amg_hier* h, int32_t reps, void* stream, amg_kernel_timing* timing);

/* The same kernel timed from HBM rather than the 256 MB Infinity Cache: the
 * library makes copies - 1 device copies of the finest level's sliced-ELL
 * column indices and weights, its diagonal (and slot map) and the step's
 * three vectors, runs one untimed round over the copies, then `reps` launches
 * back to back, launch i on copy i % copies, between two HIP events.  With
 * the copies together well above the Infinity Cache each launch streams its
 * operands from HBM.  The copies are freed before returning (this call
 * allocates and synchronizes `stream`).  1 <= copies <= 64; NOMEM if the
 * copies do not fit.  The launches are a separate kernel instance of the
 * same code, so profiles list them on their own. */
int32_t amg_time_step_rotating(amg_hier* h, int32_t reps, int32_t copies, void* stream,
                               amg_kernel_timing* timing);

/*
 * Solve nb independent systems together (Section 4's solver for each): item i
 * uses hierarchy h[i], right-hand side f[i] and initial guess / solution u[i]
 * (device pointers, n of h[i] doubles each).  A hierarchy may appear several
 * times (several right-hand sides); each repeat gets its own workspace.  All
 * items must share precision, degree, inner_steps, restart, tol and max_iter,
 * and have a coarsest level of at most 1024 rows.
 * Every cycle step is one launch covering all items that take it; each item's
 * small levels run as its own one-workgroup LDS-resident program; inner
 * products and convergence are per item on the device, converged items are
 * frozen, and one outer iteration of the whole batch is replayed as a HIP
 * graph.  An item's result does not depend on the other items of the batch.
 * infos: host array of nb records (may be NULL); solve_ms is the batch's time.
 * Returns AMG_OK if every item converged, else the first failing item's
 * status (AMG_ERR_MAXIT, AMG_ERR_BREAKDOWN) or an argument/device error.  The
 * schedule built for a set of (h, f, u) is reused while the set is unchanged.
 */
int32_t amg_solve_batch(int32_t nb, amg_hier* const* h, const double* const* f, double* const* u,
                        void* stream, amg_info* infos);

/* ---- Serving ---------------------------------------------------------------
 * Replay of an open-loop request stream.  A request names a graph by the
 * caller's graph_id and carries nrhs right-hand sides.  The graph data
 * (n, row_ptr, col, w, d; host, as for amg_setup) is read when the graph is
 * not resident (first request, or after an eviction); a request without graph
 * data for a graph that is not resident fails with AMG_ERR_ARG.
 * AMG_SERVE_BATCHED: continuous batching -- right-hand sides are admitted as
 *   slots between rounds of iters_per_step outer iterations, as they arrive
 *   and as slots (max_slots) and device memory (hbm_budget_bytes: hierarchies,
 *   slot workspaces and vectors) free up; all in-flight slots advance together
 *   through the batched executor; converged slots retire at the end of a
 *   round; new graphs are set up by a worker thread on its own stream while
 *   solves run; idle hierarchies are evicted least recently used first.
 *   Right-hand sides are admitted in submission order among requests whose
 *   graph is resident: a request waiting for its graph's setup does not hold
 *   back later requests on resident graphs.  Slot vectors come from a reused
 *   pool, so admission allocates nothing once the pool has grown.
 * AMG_SERVE_SEQUENTIAL: one right-hand side at a time in arrival order with
 *   amg_solve (the comparison mode).
 * realtime = 1: a request becomes visible at its arrival time (seconds from
 * the start of the call); 0: all requests are visible at once.
 * out: host array with one record per right-hand side, request-major
 * (sum of nrhs records); solutions go to reqs[i].u (host, nrhs * n, optional).
 * Returns AMG_OK when every request was processed (per-RHS status in out),
 * or an argument/device error. */
enum { AMG_SERVE_BATCHED = 0, AMG_SERVE_SEQUENTIAL = 1 };

typedef struct {
  double arrival_s;
  int32_t graph_id;
  int32_t n;
  const int32_t* row_ptr;  /* graph data, may be NULL for a resident graph */
  const int32_t* col;
  const double* w;
  const double* d;
  int32_t nrhs;
  const double* f;         /* host, nrhs * n values, right-hand side k at f + k n */
  double* u;               /* host output, nrhs * n values, or NULL */
} amg_request;

typedef struct {
  int32_t request;
  int32_t rhs;
  int32_t status;
  int32_t iters;
  double rel_res_true;
  double arrival_s;
  double admit_s;
  double finish_s;
} amg_completion;

typedef struct {
  amg_params params;        /* parameters of every hierarchy set up */
  double hbm_budget_bytes;  /* device memory the server may hold */
  int32_t max_slots;        /* right-hand sides in flight at once */
  int32_t mode;             /* AMG_SERVE_BATCHED or AMG_SERVE_SEQUENTIAL */
  int32_t iters_per_step;   /* outer iterations per admission round */
  int32_t realtime;
} amg_serve_cfg;

typedef struct {
  double wall_s;
  double peak_bytes;        /* largest device memory held by the server */
  int32_t evictions;
  int32_t setups;
  int32_t steps;
  int32_t max_in_flight;    /* most right-hand sides iterating at once    */
  double schedule_s;        /* serve loop time building launch schedules  */
  double admit_s;           /* serve loop time admitting right-hand sides
                               (workspace clones, copies)                 */
  double release_s;         /* serve loop time releasing memory           */
  double iterate_s;         /* serve loop time queueing and waiting for
                               rounds of outer iterations                 */
} amg_serve_stats;

/* Defaults: amg_params_default, 200e9 bytes, 256 slots, batched, 2
 * iterations per round, realtime. */
void amg_serve_cfg_default(amg_serve_cfg* cfg);

int32_t amg_serve(const amg_serve_cfg* cfg, const amg_request* reqs, int32_t nreq, amg_completion* out,
                  amg_serve_stats* stats, void* stream);

/* ---- Incremental server ------------------------------------------------------
 * The server behind amg_serve, for callers that receive requests one by one.
 * amg_server_create starts a server thread (continuous batching or the
 * sequential mode of cfg; cfg->realtime is not used: a request arrives when it
 * is submitted) that solves on `stream` and sets hierarchies up on a stream of
 * its own.  amg_server_submit copies the request's right-hand sides and graph
 * data (when given), stamps its arrival time (seconds since create) and
 * returns its ticket (0, 1, 2, ... in submission order); the solution of
 * right-hand side k goes to req->u + k n (host), which must stay valid until
 * that completion has been polled (or the server destroyed).
 * amg_server_poll moves up to `max` finished completions (oldest first;
 * `request` = ticket) into out and sets *count; with wait_s > 0 it waits up to
 * that long for the first one.  It returns the server thread's status (a
 * device error stops the server).  amg_server_destroy waits until every
 * submitted request has completed, stops the threads, frees the device memory
 * and reports stats (may be NULL); completions not yet polled are dropped.
 * Calls on one server may come from different threads. */
typedef struct amg_server amg_server;

int32_t amg_server_create(const amg_serve_cfg* cfg, void* stream, amg_server** out);
int32_t amg_server_submit(amg_server* srv, const amg_request* req, int32_t* ticket);
int32_t amg_server_poll(amg_server* srv, amg_completion* out, int32_t max, double wait_s, int32_t* count);
int32_t amg_server_destroy(amg_server* srv, amg_serve_stats* stats);

/* ---- Level inspection and single steps (tests and diagnostics) ------------
 * The single steps below (all but amg_apply_cycle) need an AMG_FP64
 * hierarchy (AMG_ERR_ARG otherwise); each synchronizes `stream` before it
 * returns. */

/* Export level l (host pointers, sized from amg_describe): off-diagonal CSR
 * (row_ptr n+1, col nnz, W nnz), d and D (n each), and for l < levels-1 the
 * aggregate map agg (n entries, values in [0, n_{l+1})).  Any pointer may be
 * NULL to skip that array. */
int32_t amg_level_export(const amg_hier* h, int32_t level, int32_t* row_ptr, int32_t* col,
                         double* W, double* d, double* D, int32_t* agg);

/* y = q_m(A_l) r (Section 3 smoother, m matrix-vector products); device
 * pointers of n_l doubles; level < levels-1. */
int32_t amg_apply_smoother(amg_hier* h, int32_t level, const double* r, double* y, void* stream);

/* s = f - A_l x; device pointers of n_l doubles. */
int32_t amg_apply_residual(amg_hier* h, int32_t level, const double* f, const double* x,
                           double* s, void* stream);

/* b = P^T s (sum over each aggregate): s has n_l, b has n_{l+1} doubles. */
int32_t amg_apply_restrict(amg_hier* h, int32_t level, const double* s, double* b, void* stream);

/* x += P e (each vertex adds its aggregate's value): e has n_{l+1}, x n_l. */
int32_t amg_apply_prolong(amg_hier* h, int32_t level, const double* e, double* x, void* stream);

/* x = A_L^{-1} b on the coarsest level by the Cholesky factor. */
int32_t amg_apply_coarse(amg_hier* h, const double* b, double* x, void* stream);

/* z = Kcycle(0, r): one application of the preconditioner on the finest level. */
int32_t amg_apply_cycle(amg_hier* h, const double* r, double* z, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AMG_H */
