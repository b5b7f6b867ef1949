// Host-side validation of the problem data of eq. (prob) and of the solver
// parameters.  Runs before any device call so that invalid input is reported
// the same way with or without a GPU.
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "amg.h"

namespace amg {

namespace {

double smoother_error(int m, double kappa) {
  const double sk = std::sqrt(kappa);
  const double delta = (sk - 1.0) / (sk + 1.0);
  return std::pow(delta, m) * (kappa - 1.0) / 2.0;
}

}  // namespace

// Section 3: E_m = delta^m (kappa - 1) / 2 decreases in m; the smallest m
// meeting both the damping requirement (E_m <= rho) and E_m < 1.
int32_t resolved_degree(const amg_params& p) {
  if (p.degree >= 0) return p.degree;
  int m = 0;
  while (m < 64 && !(smoother_error(m, p.lambda0_ratio) <= p.smoother_rho && smoother_error(m, p.lambda0_ratio) < 1.0))
    ++m;
  return m;
}

int32_t validate_params(const amg_params& p, std::string& msg) {
  if (p.degree < -1 || p.degree > 64) { msg = "degree out of range [-1, 64]"; return AMG_ERR_ARG; }
  if (p.degree == -1 && !(p.smoother_rho > 0.0 && p.smoother_rho <= 1.0)) {
    msg = "smoother_rho must lie in (0, 1] for degree -1";
    return AMG_ERR_ARG;
  }
  if (p.agg_size < 2 || p.agg_size > (1 << 12)) { msg = "agg_size out of range [2, 4096]"; return AMG_ERR_ARG; }
  if (p.coarse_max < 1) { msg = "coarse_max must be >= 1"; return AMG_ERR_ARG; }
  if (!(p.lambda0_ratio > 1.0) || !std::isfinite(p.lambda0_ratio)) { msg = "lambda0_ratio must be > 1"; return AMG_ERR_ARG; }
  if (p.inner_steps < 1 || p.inner_steps > 8) { msg = "inner_steps out of range [1, 8]"; return AMG_ERR_ARG; }
  if (p.restart < 1 || p.restart > 8) { msg = "restart out of range [1, 8]"; return AMG_ERR_ARG; }
  if (!(p.tol > 0.0) || !(p.tol < 1.0)) { msg = "tol must lie in (0, 1)"; return AMG_ERR_ARG; }
  if (p.max_iter < 1) { msg = "max_iter must be >= 1"; return AMG_ERR_ARG; }
  if (p.precision != AMG_FP64 && p.precision != AMG_MIXED) { msg = "unknown precision"; return AMG_ERR_ARG; }
  if (p.match_key != AMG_KEY_NORMALIZED && p.match_key != AMG_KEY_RAW) { msg = "unknown match_key"; return AMG_ERR_ARG; }
  if (p.max_coarsest < 1 || p.max_coarsest > 4096) { msg = "max_coarsest out of range [1, 4096]"; return AMG_ERR_ARG; }
  if (!(p.stagnation > 0.0) || !(p.stagnation < 1.0)) { msg = "stagnation must lie in (0, 1)"; return AMG_ERR_ARG; }
  if (p.tail_rows < 0) { msg = "tail_rows must be >= 0"; return AMG_ERR_ARG; }
  if (p.autotune != 0 && p.autotune != 1) { msg = "autotune must be 0 or 1"; return AMG_ERR_ARG; }
  if (p.slice_height != 8 && p.slice_height != 16 && p.slice_height != 32 && p.slice_height != 64) {
    msg = "slice_height must be 8, 16, 32 or 64";
    return AMG_ERR_ARG;
  }
  if (p.lanes_per_row != 1 && p.lanes_per_row != 2 && p.lanes_per_row != 4) {
    msg = "lanes_per_row must be 1, 2 or 4";
    return AMG_ERR_ARG;
  }
  if (p.sort_rows != 0 && p.sort_rows != 1) { msg = "sort_rows must be 0 or 1"; return AMG_ERR_ARG; }
  if (p.fuse != 0 && p.fuse != 1) { msg = "fuse must be 0 or 1"; return AMG_ERR_ARG; }
  if (p.cycle != AMG_CYCLE_K && p.cycle != AMG_CYCLE_AMLI) {
    msg = "cycle must be AMG_CYCLE_K or AMG_CYCLE_AMLI";
    return AMG_ERR_ARG;
  }
  if (p.aggregation != AMG_AGG_MATCHING && p.aggregation != AMG_AGG_MIS) {
    msg = "aggregation must be AMG_AGG_MATCHING or AMG_AGG_MIS";
    return AMG_ERR_ARG;
  }
  if (p.mis_distance < 1 || p.mis_distance > 8) { msg = "mis_distance must be in [1, 8]"; return AMG_ERR_ARG; }
  if (p.neumann != 0 && p.neumann != 1) { msg = "neumann must be 0 or 1"; return AMG_ERR_ARG; }
  if (p.stop != AMG_STOP_RESIDUAL && p.stop != AMG_STOP_ENERGY) {
    msg = "stop must be AMG_STOP_RESIDUAL or AMG_STOP_ENERGY";
    return AMG_ERR_ARG;
  }
  if (p.cycle == AMG_CYCLE_AMLI && p.inner_steps != 2) {
    msg = "the AMLI cycle is a W-cycle: inner_steps must be 2";
    return AMG_ERR_ARG;
  }
  if (p.tie_break != AMG_TIE_INDEX && p.tie_break != AMG_TIE_HASH) {
    msg = "tie_break must be AMG_TIE_INDEX or AMG_TIE_HASH";
    return AMG_ERR_ARG;
  }
  // Smoother damping on [lambda0, lambda1]: E_m = delta^m (kappa - 1) / 2 must be < 1.
  const double kappa = p.lambda0_ratio;
  const double sk = std::sqrt(kappa);
  const double delta = (sk - 1.0) / (sk + 1.0);
  const double Em = std::pow(delta, resolved_degree(p)) * (kappa - 1.0) / 2.0;
  if (!(Em < 1.0)) { msg = "smoother degree too low for lambda0_ratio: E_m >= 1"; return AMG_ERR_DEGREE; }
  return AMG_OK;
}

// CSR checks: sizes, ranges, strictly increasing columns, no self loops,
// positive finite weights stored symmetrically with identical values,
// non-negative finite d with at least one positive entry (unless
// allow_singular), connectivity.
int32_t validate_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                       const double* d, std::string& msg, bool allow_singular) {
  if (n < 1) { msg = "n must be >= 1"; return AMG_ERR_ARG; }
  if (!row_ptr || !d) { msg = "null row_ptr or d"; return AMG_ERR_ARG; }
  if (row_ptr[0] != 0) { msg = "row_ptr[0] != 0"; return AMG_ERR_GRAPH; }
  for (int32_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) { msg = "row_ptr decreasing at row " + std::to_string(i); return AMG_ERR_GRAPH; }
  const int64_t nnz = row_ptr[n];
  if (nnz > 0 && (!col || !w)) { msg = "null col or w"; return AMG_ERR_ARG; }
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col[k];
      if (j < 0 || j >= n) { msg = "column out of range in row " + std::to_string(i); return AMG_ERR_GRAPH; }
      if (j == i) { msg = "self loop at row " + std::to_string(i); return AMG_ERR_GRAPH; }
      if (k > row_ptr[i] && col[k - 1] >= j) { msg = "columns not strictly increasing in row " + std::to_string(i); return AMG_ERR_GRAPH; }
      if (!(w[k] > 0.0) || !std::isfinite(w[k])) { msg = "weight not positive and finite in row " + std::to_string(i); return AMG_ERR_GRAPH; }
    }
  }
  // symmetry: (i, j, w) must have a partner (j, i, w) with the identical value
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const int32_t j = col[k];
      int32_t lo = row_ptr[j], hi = row_ptr[j + 1];
      while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (col[mid] < i) lo = mid + 1; else hi = mid;
      }
      if (lo == row_ptr[j + 1] || col[lo] != i || w[lo] != w[k]) {
        msg = "asymmetric entry (" + std::to_string(i) + ", " + std::to_string(j) + ")";
        return AMG_ERR_GRAPH;
      }
    }
  }
  bool any_d = false;
  for (int32_t i = 0; i < n; ++i) {
    if (!(d[i] >= 0.0) || !std::isfinite(d[i])) { msg = "d not non-negative and finite at " + std::to_string(i); return AMG_ERR_GRAPH; }
    any_d = any_d || d[i] > 0.0;
  }
  // connectivity by breadth-first search from vertex 0
  std::vector<int32_t> queue;
  queue.reserve(n);
  std::vector<uint8_t> seen(n, 0);
  queue.push_back(0);
  seen[0] = 1;
  for (size_t h = 0; h < queue.size(); ++h) {
    const int32_t v = queue[h];
    for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      const int32_t u = col[k];
      if (!seen[u]) { seen[u] = 1; queue.push_back(u); }
    }
  }
  if ((int32_t)queue.size() != n) { msg = "graph is not connected"; return AMG_ERR_DISCONNECTED; }
  if (!any_d && !allow_singular) { msg = "all d_i are zero: A is singular (set neumann = 1)"; return AMG_ERR_SINGULAR; }
  return AMG_OK;
}

}  // namespace amg
