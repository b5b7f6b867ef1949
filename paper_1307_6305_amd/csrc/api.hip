// C ABI (include/amg.h): argument checking, handle lifetime, dispatch to the
// setup and solve translation units.
#include <cstring>
#include <string>

#include "hier.h"

namespace amg {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& m) { g_last_error = m; }

int32_t dalloc(amg_hier* h, void** p, size_t bytes) {
  if (h->arena) {
    const size_t at = (h->arena_used + 255) & ~size_t(255);
    if (at + bytes <= h->arena_cap) {
      *p = h->arena + at;
      h->arena_used = at + bytes;
      return AMG_OK;
    }
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    set_last_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    *p = nullptr;
    return e == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;
  }
  h->allocs.push_back(q);
  h->bytes += bytes;
  *p = q;
  return AMG_OK;
}

// the parent's workspace, with room for the 256-byte alignment of each of
// its buffers (several per level)
size_t clone_bytes_of(const amg_hier* h) { return h->ws_bytes + 256 * (32 * (size_t)h->lv.size() + 64); }

int32_t make_clone(amg_hier* h, amg_hier** out, hipStream_t s) {
  amg_hier* c = new amg_hier();
  c->p = h->p;
  c->device = h->device;
  c->mixed = h->mixed;
  c->lv = h->lv;
  c->L = h->L;
  c->chol = h->chol;
  c->chol_inv = h->chol_inv;
  c->chol_invT = h->chol_invT;
  c->nL = h->nL;
  c->desc = h->desc;
  c->amli_a = h->amli_a;
  c->amli_g0 = h->amli_g0;
  c->amli_g1 = h->amli_g1;
  c->parent = h;
  // one arena; a clone that outgrows it falls back to separate allocations
  const size_t cap = clone_bytes_of(h);
  void* a = nullptr;
  if (hipMalloc(&a, cap) == hipSuccess) {
    c->arena = static_cast<char*>(a);
    c->arena_cap = cap;
    c->bytes += cap;
  } else {
    (void)hipGetLastError();
  }
  const int32_t st = prepare_solve(c, s);
  if (st != AMG_OK) {
    free_clone(c);
    return st;
  }
  *out = c;
  return AMG_OK;
}

// The caller guarantees that no queued work still uses the clone (the server
// and the batched solve synchronize their stream before releasing one); the
// clone's own graphs ran on its graph stream.  (hipFree still waits for the
// device to drain: a release costs a device-wide wait, which is why the server
// reuses idle clones rather than freeing them.)
void free_clone(amg_hier* c) {
  if (!c) return;
  if (c->graph_stream) (void)hipStreamSynchronize(c->graph_stream);
  destroy_graphs(c);
  if (c->graph_stream) (void)hipStreamDestroy(c->graph_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->arena) (void)hipFree(c->arena);
  if (c->host_scal) (void)hipHostFree(c->host_scal);
  delete c;
}

}  // namespace amg

namespace {

int32_t check_device() {
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count < 1) {
    amg::set_last_error(e != hipSuccess ? std::string("hipGetDeviceCount: ") + hipGetErrorString(e)
                                        : std::string("no HIP device"));
    return AMG_ERR_DEVICE;
  }
  return AMG_OK;
}

int32_t check_level(const amg_hier* h, int32_t level, bool allow_coarsest) {
  if (!h) { amg::set_last_error("null handle"); return AMG_ERR_ARG; }
  const int top = allow_coarsest ? h->L : h->L - 1;
  if (level < 0 || level > top) { amg::set_last_error("level out of range"); return AMG_ERR_ARG; }
  return AMG_OK;
}

int32_t check_fp64_steps(const amg_hier* h) {
  if (h->mixed) {
    amg::set_last_error("single-step entry points need an FP64 hierarchy");
    return AMG_ERR_ARG;
  }
  return AMG_OK;
}

int32_t sync_status(hipStream_t s) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    amg::set_last_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return AMG_ERR_DEVICE;
  }
  return AMG_OK;
}

}  // namespace

extern "C" {

void amg_params_default(amg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->degree = 4;
  p->agg_size = 4;
  p->coarse_max = 64;
  p->lambda0_ratio = 10.0;
  p->inner_steps = 2;
  p->restart = 5;
  p->tol = 1e-8;
  p->max_iter = 200;
  p->precision = AMG_FP64;
  p->match_key = AMG_KEY_NORMALIZED;
  p->max_coarsest = 2048;
  p->stagnation = 0.9;
  p->use_graph = 1;
  p->tail_rows = 4096;
  p->autotune = 1;
  p->slice_height = 64;
  p->lanes_per_row = 1;
  p->sort_rows = 0;
  p->tie_break = AMG_TIE_INDEX;
  p->fuse = 1;
  p->smoother_rho = 0.33;
  p->cycle = AMG_CYCLE_K;
  p->aggregation = AMG_AGG_MATCHING;
  p->mis_distance = 4;
  p->neumann = 0;
  p->stop = AMG_STOP_RESIDUAL;
}

const char* amg_strerror(int32_t s) {
  switch (s) {
    case AMG_OK: return "ok";
    case AMG_ERR_ARG: return "invalid argument";
    case AMG_ERR_GRAPH: return "malformed graph";
    case AMG_ERR_DISCONNECTED: return "graph not connected";
    case AMG_ERR_SINGULAR: return "singular operator";
    case AMG_ERR_DEGREE: return "smoother degree too low";
    case AMG_ERR_COARSEN: return "coarsening stagnated";
    case AMG_ERR_NOMEM: return "out of device memory";
    case AMG_ERR_DEVICE: return "device error";
    case AMG_ERR_BREAKDOWN: return "flexible CG breakdown";
    case AMG_ERR_MAXIT: return "iteration limit reached";
    case AMG_ERR_BUDGET: return "over memory budget";
    default: return "unknown status";
  }
}

const char* amg_last_error(void) { return amg::g_last_error.c_str(); }

int32_t amg_setup(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w, const double* d,
                  const amg_params* params, void* stream, amg_hier** out) {
  if (!out) { amg::set_last_error("null output handle"); return AMG_ERR_ARG; }
  *out = nullptr;
  amg_params p;
  if (params) p = *params; else amg_params_default(&p);
  std::string msg;
  int32_t st = amg::validate_params(p, msg);
  if (st != AMG_OK) { amg::set_last_error(msg); return st; }
  p.degree = amg::resolved_degree(p);
  st = amg::validate_graph(n, row_ptr, col, w, d, msg, p.neumann != 0);
  if (st != AMG_OK) { amg::set_last_error(msg); return st; }
  AMG_TRY(check_device());
  amg_hier* h = new amg_hier();
  h->p = p;
  h->mixed = p.precision == AMG_MIXED;
  (void)hipGetDevice(&h->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = amg::build_hierarchy(h, n, row_ptr, col, w, d, s);
  if (st == AMG_OK) st = amg::prepare_solve(h, s);
  if (st != AMG_OK) {
    amg_free(h);
    return st;
  }
  *out = h;
  return AMG_OK;
}

void amg_free(amg_hier* h) {
  if (!h) return;
  amg::drop_batches_using(h);
  (void)hipDeviceSynchronize();
  amg::destroy_graphs(h);
  if (h->graph_stream) (void)hipStreamDestroy(h->graph_stream);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->host_scal) (void)hipHostFree(h->host_scal);
  delete h;
}

int32_t amg_describe(const amg_hier* h, amg_hier_desc* out) {
  if (!h || !out) { amg::set_last_error("null argument"); return AMG_ERR_ARG; }
  *out = h->desc;
  out->device_bytes = (double)h->bytes;
  return AMG_OK;
}

int32_t amg_solve(amg_hier* h, const double* f, double* u, void* stream, amg_info* info) {
  if (!h || !f || !u) { amg::set_last_error("null argument"); return AMG_ERR_ARG; }
  return amg::solve(h, f, u, static_cast<hipStream_t>(stream), info);
}

int32_t amg_solve_noalloc(amg_hier* h, const double* f, double* u, void* stream, amg_info* info) {
  if (!h || !f || !u) { amg::set_last_error("null argument"); return AMG_ERR_ARG; }
  return amg::solve_noalloc(h, f, u, static_cast<hipStream_t>(stream), info);
}

int32_t amg_solve_batch(int32_t nb, amg_hier* const* h, const double* const* f, double* const* u, void* stream,
                        amg_info* infos) {
  if (nb < 1 || !h || !f || !u) { amg::set_last_error("invalid argument"); return AMG_ERR_ARG; }
  for (int32_t i = 0; i < nb; ++i)
    if (!h[i] || !f[i] || !u[i]) { amg::set_last_error("null item " + std::to_string(i)); return AMG_ERR_ARG; }
  return amg::solve_batch(nb, h, f, u, static_cast<hipStream_t>(stream), infos);
}

void amg_serve_cfg_default(amg_serve_cfg* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  amg_params_default(&c->params);
  c->hbm_budget_bytes = 200e9;
  c->max_slots = 256;
  c->mode = AMG_SERVE_BATCHED;
  c->iters_per_step = 2;
  c->realtime = 1;
}

namespace {

int32_t check_serve_cfg(const amg_serve_cfg* cfg) {
  if (!cfg) { amg::set_last_error("null configuration"); return AMG_ERR_ARG; }
  if (cfg->mode != AMG_SERVE_BATCHED && cfg->mode != AMG_SERVE_SEQUENTIAL) {
    amg::set_last_error("unknown serve mode");
    return AMG_ERR_ARG;
  }
  if (!(cfg->hbm_budget_bytes > 0) || cfg->max_slots < 1) {
    amg::set_last_error("budget and max_slots must be positive");
    return AMG_ERR_ARG;
  }
  std::string msg;
  const int32_t pst = amg::validate_params(cfg->params, msg);
  if (pst != AMG_OK) {
    amg::set_last_error(msg);
    return pst;
  }
  if (cfg->params.stop != AMG_STOP_RESIDUAL) {
    amg::set_last_error("the served form uses the residual stopping test (AMG_STOP_RESIDUAL) only");
    return AMG_ERR_ARG;
  }
  return AMG_OK;
}

int32_t check_request(const amg_request& q, int32_t i) {
  if (q.n < 1 || q.nrhs < 1 || !q.f) {
    amg::set_last_error("request " + std::to_string(i) + ": n, nrhs and f are required");
    return AMG_ERR_ARG;
  }
  if (q.row_ptr && (!q.col || !q.w || !q.d)) {
    amg::set_last_error("request " + std::to_string(i) + ": graph data needs row_ptr, col, w and d");
    return AMG_ERR_ARG;
  }
  return AMG_OK;
}

}  // namespace

int32_t amg_serve(const amg_serve_cfg* cfg, const amg_request* reqs, int32_t nreq, amg_completion* out,
                  amg_serve_stats* stats, void* stream) {
  if (!reqs || nreq < 1 || !out) { amg::set_last_error("invalid argument"); return AMG_ERR_ARG; }
  AMG_TRY(check_serve_cfg(cfg));
  for (int32_t i = 0; i < nreq; ++i) AMG_TRY(check_request(reqs[i], i));
  AMG_TRY(check_device());
  return amg::serve(*cfg, reqs, nreq, out, stats, static_cast<hipStream_t>(stream));
}

int32_t amg_server_create(const amg_serve_cfg* cfg, void* stream, amg_server** out) {
  if (!out) { amg::set_last_error("null output handle"); return AMG_ERR_ARG; }
  *out = nullptr;
  AMG_TRY(check_serve_cfg(cfg));
  AMG_TRY(check_device());
  void* p = nullptr;
  AMG_TRY(amg::server_create(*cfg, static_cast<hipStream_t>(stream), &p));
  *out = static_cast<amg_server*>(p);
  return AMG_OK;
}

int32_t amg_server_submit(amg_server* srv, const amg_request* req, int32_t* ticket) {
  if (!srv || !req) { amg::set_last_error("null argument"); return AMG_ERR_ARG; }
  AMG_TRY(check_request(*req, 0));
  return amg::server_submit(srv, *req, ticket);
}

int32_t amg_server_poll(amg_server* srv, amg_completion* out, int32_t max, double wait_s, int32_t* count) {
  if (!srv || !out || max < 1 || !count) { amg::set_last_error("invalid argument"); return AMG_ERR_ARG; }
  return amg::server_poll(srv, out, max, wait_s, count);
}

int32_t amg_server_destroy(amg_server* srv, amg_serve_stats* stats) {
  if (!srv) return AMG_OK;
  return amg::server_destroy(srv, stats);
}

int32_t amg_time_step(amg_hier* h, int32_t reps, void* stream, amg_kernel_timing* timing) {
  if (!h || !timing || reps < 1) { amg::set_last_error("invalid argument"); return AMG_ERR_ARG; }
  if (h->L < 1) { amg::set_last_error("the finest level is not smoothed in a one-level hierarchy"); return AMG_ERR_ARG; }
  return amg::time_step(h, reps, static_cast<hipStream_t>(stream), timing);
}

int32_t amg_time_step_rotating(amg_hier* h, int32_t reps, int32_t copies, void* stream, amg_kernel_timing* timing) {
  if (!h || !timing || reps < 1 || copies < 1 || copies > 64) {
    amg::set_last_error("invalid argument (reps >= 1, 1 <= copies <= 64)");
    return AMG_ERR_ARG;
  }
  if (h->L < 1) { amg::set_last_error("the finest level is not smoothed in a one-level hierarchy"); return AMG_ERR_ARG; }
  return amg::time_step_rotating(h, reps, copies, static_cast<hipStream_t>(stream), timing);
}

int32_t amg_level_export(const amg_hier* h, int32_t level, int32_t* row_ptr, int32_t* col, double* W, double* d,
                         double* D, int32_t* agg) {
  AMG_TRY(check_level(h, level, true));
  const amg::Level& lv = h->lv[level];
  AMG_HIP(hipDeviceSynchronize());
  if (row_ptr) AMG_HIP(hipMemcpy(row_ptr, lv.row_ptr, sizeof(int32_t) * (lv.n + 1), hipMemcpyDeviceToHost));
  if (col && lv.nnz) AMG_HIP(hipMemcpy(col, lv.col, sizeof(int32_t) * lv.nnz, hipMemcpyDeviceToHost));
  if (W && lv.nnz) AMG_HIP(hipMemcpy(W, lv.W, sizeof(double) * lv.nnz, hipMemcpyDeviceToHost));
  if (d) AMG_HIP(hipMemcpy(d, lv.d, sizeof(double) * lv.n, hipMemcpyDeviceToHost));
  if (D) AMG_HIP(hipMemcpy(D, lv.D, sizeof(double) * lv.n, hipMemcpyDeviceToHost));
  if (agg && level < h->L) AMG_HIP(hipMemcpy(agg, lv.agg, sizeof(int32_t) * lv.n, hipMemcpyDeviceToHost));
  return AMG_OK;
}

int32_t amg_apply_smoother(amg_hier* h, int32_t level, const double* r, double* y, void* stream) {
  AMG_TRY(check_level(h, level, false));
  AMG_TRY(check_fp64_steps(h));
  if (!r || !y) return AMG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_smoother(h, level, r, y, s));
  return sync_status(s);
}

int32_t amg_apply_residual(amg_hier* h, int32_t level, const double* f, const double* x, double* s_out,
                           void* stream) {
  AMG_TRY(check_level(h, level, false));
  AMG_TRY(check_fp64_steps(h));
  if (!f || !x || !s_out) return AMG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_residual(h, level, f, x, s_out, s));
  return sync_status(s);
}

int32_t amg_apply_restrict(amg_hier* h, int32_t level, const double* sv, double* b, void* stream) {
  AMG_TRY(check_level(h, level, false));
  AMG_TRY(check_fp64_steps(h));
  if (!sv || !b) return AMG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_restrict(h, level, sv, b, s));
  return sync_status(s);
}

int32_t amg_apply_prolong(amg_hier* h, int32_t level, const double* e, double* x, void* stream) {
  AMG_TRY(check_level(h, level, false));
  AMG_TRY(check_fp64_steps(h));
  if (!e || !x) return AMG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_prolong(h, level, e, x, s));
  return sync_status(s);
}

int32_t amg_apply_coarse(amg_hier* h, const double* b, double* x, void* stream) {
  if (!h || !b || !x) return AMG_ERR_ARG;
  AMG_TRY(check_fp64_steps(h));
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_coarse(h, b, x, s));
  return sync_status(s);
}

int32_t amg_apply_cycle(amg_hier* h, const double* r, double* z, void* stream) {
  if (!h || !r || !z) return AMG_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  AMG_TRY(amg::step_cycle(h, r, z, s));
  return sync_status(s);
}

}  // extern "C"
