// The hierarchy object behind the opaque amg_hier handle, and the interfaces
// between the setup, solve and API translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"

struct amg_hier {
  amg_params p{};
  // a workspace clone shares the levels of `parent` and owns only its solve
  // workspace (several right-hand sides of one hierarchy in a batch)
  const amg_hier* parent = nullptr;
  int device = 0;
  bool mixed = false;
  std::vector<amg::Level> lv;  // finest first; lv.back() is the coarsest
  int L = 0;                   // index of the coarsest level
  // coarsest level: dense Cholesky factor (row-major, lower triangle used)
  double* chol = nullptr;
  double* chol_inv = nullptr;   // L^-1 (row-major), when nL <= 1024
  double* chol_invT = nullptr;  // (L^-1)^T
  int32_t nL = 0;

  // tail program: the inner solve of level tail_level (and all below) run by
  // one workgroup (0 = no tail)
  int tail_level = 0;
  int tail_nops = 0;
  size_t tail_lds_bytes = 0;           // dynamic LDS of the tail kernel
  int tail_threads = 0;                // workgroup size of the tail kernel
  const void* tail_prog = nullptr;     // kernel argument block (host copy)
  std::vector<char> tail_prog_storage;

  // Solve workspace.  `vt` buffers hold the cycle's vector type (double, or
  // float in mixed precision); per level: A, B (smoother recurrence), S
  // (residual); rhs/sol of the level's inner solve; Z[k], Q[k] directions.
  struct Work {
    void* A = nullptr;
    void* B = nullptr;
    void* S = nullptr;
    void* rhs = nullptr;
    void* sol = nullptr;
    void* Z[8] = {};
    void* Q[8] = {};
    // launch-bound levels with two inner steps: the right-hand side after
    // step 0 and the direction of step 1 (updates folded into later kernels)
    void* rhs2 = nullptr;
    void* P1 = nullptr;
    // launch-bound levels: aggregate-to-block map of the fused residual +
    // restriction, and the row-to-slot map of a sorted layout
    void* agg_blk = nullptr;
    int n_agg_blk = 0;
    void* slot_of_row = nullptr;
  };
  std::vector<Work> ws;
  // outer flexible CG (always FP64, finest level)
  double* r = nullptr;
  void* z = nullptr;  // cycle output (cycle vector type)
  double* P[8] = {};
  double* Qo[8] = {};
  double* tmp = nullptr;

  double* scal = nullptr;       // device scalar area (see solve.hip for the slots)
  double* partials = nullptr;   // grid-reduction partial sums
  unsigned* counter = nullptr;  // grid-reduction arrival counter
  double* host_scal = nullptr;  // pinned host mirror of a few scalars
  int max_blocks = 0;
  int last_block_max = 32;

  // replayable outer iterations (one per position in the restart window)
  bool graphs_ready = false;
  hipGraphExec_t iter_exec[8] = {};
  hipStream_t graph_stream = nullptr;  // stream the graphs were captured on
  const void* graph_u = nullptr;       // solution pointer baked into the graphs
  hipEvent_t iter_ev[2] = {};          // completion of the outer iterations in flight

  // stationary AMLI cycle: per level, the estimated lambda_min(B_l A_l) and
  // the coarse-correction polynomial g0 + g1 t (levels 1 .. L-1)
  std::vector<double> amli_a, amli_g0, amli_g1;

  amg_hier_desc desc{};
  std::vector<void*> allocs;
  size_t bytes = 0;     // device bytes owned (allocs and arena)
  // A workspace clone takes its buffers from one block (one allocation and
  // one release per clone: each release waits for the device to drain).
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  size_t ws_bytes = 0;  // of which the solve workspace (what a clone costs)
};

namespace amg {

int32_t validate_params(const amg_params& p, std::string& msg);
// The smoother degree in use: p.degree, or for -1 the smallest m with
// E_m <= p.smoother_rho and E_m < 1 (valid parameters only).
int32_t resolved_degree(const amg_params& p);
// allow_singular: d = 0 everywhere is accepted (pure Neumann problem).
int32_t validate_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                       const double* d, std::string& msg, bool allow_singular = false);

// Device allocation owned by the hierarchy (freed by amg_free).
int32_t dalloc(amg_hier* h, void** p, size_t bytes);
template <typename T>
int32_t dalloc(amg_hier* h, T** p, size_t count) {
  return dalloc(h, reinterpret_cast<void**>(p), count * sizeof(T) + 16);
}

struct Level;
// Mean time of one storing Chebyshev step on `lv` (its current layout), on
// zero vectors wk, wb, y of the level's cycle precision (layout autotuner).
int32_t time_cheb_layout(const Level& lv, bool mixed, void* wk, void* wb, void* y, hipStream_t s, float* ms);

int32_t build_hierarchy(amg_hier* h, int32_t n, const int32_t* row_ptr, const int32_t* col,
                        const double* w, const double* d, hipStream_t s);
int32_t prepare_solve(amg_hier* h, hipStream_t s);
void destroy_graphs(amg_hier* h);

// single steps (FP64 device vectors at the boundary)
int32_t step_smoother(amg_hier* h, int l, const double* r, double* y, hipStream_t s);
int32_t step_residual(amg_hier* h, int l, const double* f, const double* x, double* out, hipStream_t s);
int32_t step_restrict(amg_hier* h, int l, const double* sv, double* b, hipStream_t s);
int32_t step_prolong(amg_hier* h, int l, const double* e, double* x, hipStream_t s);
int32_t step_coarse(amg_hier* h, const double* b, double* x, hipStream_t s);
int32_t step_cycle(amg_hier* h, const double* r, double* z, hipStream_t s);

int32_t solve(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info);
// The same solve with its reduction scratch in a static device array (no
// allocation, no graphs, no events); finest levels up to noalloc_max_rows().
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
int32_t solve_noalloc(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info);
size_t noalloc_max_rows();

// batched solves (batch.hip)
int32_t solve_batch(int nb, amg_hier* const* hs, const double* const* f, double* const* u, hipStream_t s,
                    amg_info* infos);
void drop_batches_using(const amg_hier* h);
// Device bytes a clone of h takes (its workspace arena).
size_t clone_bytes_of(const amg_hier* h);
int32_t make_clone(amg_hier* h, amg_hier** out, hipStream_t s);
void free_clone(amg_hier* c);

// serving (serve.hip)
int32_t serve(const amg_serve_cfg& cfg, const amg_request* reqs, int32_t nreq, amg_completion* out,
              amg_serve_stats* stats, hipStream_t s);
int32_t server_create(const amg_serve_cfg& cfg, hipStream_t s, void** out);
int32_t server_submit(void* srv, const amg_request& q, int32_t* ticket);
int32_t server_poll(void* srv, amg_completion* out, int32_t max, double wait_s, int32_t* count);
int32_t server_destroy(void* srv, amg_serve_stats* stats);
int32_t time_step(amg_hier* h, int reps, hipStream_t s, amg_kernel_timing* t);
int32_t time_step_rotating(amg_hier* h, int reps, int copies, hipStream_t s, amg_kernel_timing* t);

}  // namespace amg
