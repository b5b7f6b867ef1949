// Randomized check of the host-side graph validation (problem data of
// eq. (prob)): random connected graphs in CSR form, each left valid or given
// exactly one defect, must be classified with the status the C ABI documents
// for that defect.  Built by tests/test_validate_fuzz.py with the address and
// undefined-behaviour sanitizers, so a read outside the caller's arrays fails
// the run.  Prints one line per defect kind: "<kind> <trials>".
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <string>
#include <utility>
#include <vector>

#include "amg.h"

namespace amg {
int32_t validate_graph(int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w, const double* d,
                       std::string& msg, bool allow_singular);
}

namespace {

enum Kind {
  K_VALID, K_COL_RANGE, K_SELF_LOOP, K_UNSORTED, K_WEIGHT_NONPOS, K_WEIGHT_NAN, K_ASYMMETRIC, K_D_NEGATIVE,
  K_D_NAN, K_ROW_PTR_DECREASING, K_ROW_PTR_START, K_DISCONNECTED, K_ALL_D_ZERO, K_ALL_D_ZERO_ALLOWED, K_COUNT
};
const char* kNames[K_COUNT] = {"valid",        "col_range",   "self_loop",  "unsorted",           "weight_nonpos",
                               "weight_nan",   "asymmetric",  "d_negative", "d_nan",              "row_ptr_decreasing",
                               "row_ptr_start", "disconnected", "all_d_zero", "all_d_zero_allowed"};

struct Csr {
  int n = 0;
  std::vector<int32_t> rp, col;
  std::vector<double> w, d;
};

// Symmetric CSR with sorted rows from an undirected edge list (no duplicates).
Csr build(int n, const std::vector<std::pair<int, int>>& edges, std::mt19937& rng) {
  std::vector<std::vector<std::pair<int, double>>> adj(n);
  for (const auto& e : edges) {
    const double we = 0.25 * (1 + rng() % 16);
    adj[e.first].push_back({e.second, we});
    adj[e.second].push_back({e.first, we});
  }
  Csr g;
  g.n = n;
  g.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    for (const auto& a : adj[i]) {
      g.col.push_back(a.first);
      g.w.push_back(a.second);
    }
    g.rp[i + 1] = (int32_t)g.col.size();
  }
  g.d.assign(n, 0.0);
  g.d[rng() % n] = 1.0 + rng() % 3;
  return g;
}

// A random connected graph: a random tree plus extra edges (components > 1
// joins nothing across the split point).
Csr random_graph(int n, int components, std::mt19937& rng) {
  std::vector<std::pair<int, int>> edges;
  const int split = components > 1 ? 1 + (int)(rng() % (n - 1)) : n;
  auto comp = [&](int v) { return v < split ? 0 : 1; };
  for (int v = 1; v < n; ++v) {
    if (v == split) continue;  // first vertex of the second component
    const int lo = comp(v) == 0 ? 0 : split;
    edges.push_back({lo + (int)(rng() % (v - lo)), v});
  }
  const int extra = (int)(rng() % (2 * n + 1));
  for (int t = 0; t < extra; ++t) {
    const int a = (int)(rng() % n), b = (int)(rng() % n);
    if (a == b || comp(a) != comp(b)) continue;
    const std::pair<int, int> e{std::min(a, b), std::max(a, b)};
    bool dup = false;
    for (const auto& f : edges) dup = dup || (std::min(f.first, f.second) == e.first && std::max(f.first, f.second) == e.second);
    if (!dup) edges.push_back(e);
  }
  return build(n, edges, rng);
}

int row_of(const Csr& g, int k) {
  return (int)(std::upper_bound(g.rp.begin(), g.rp.end(), k) - g.rp.begin()) - 1;
}

}  // namespace

int main(int argc, char** argv) {
  const int trials = argc > 1 ? std::atoi(argv[1]) : 20000;
  std::mt19937 rng(12345);
  int seen[K_COUNT] = {0};
  for (int t = 0; t < trials; ++t) {
    const Kind kind = (Kind)(t % K_COUNT);
    // at least three vertices where a row with two entries is needed (a tree
    // on three or more vertices has a vertex of degree two)
    const int n = (kind == K_UNSORTED ? 3 : 2) + (int)(rng() % 22);
    Csr g = random_graph(n, kind == K_DISCONNECTED ? 2 : 1, rng);
    const int nnz = (int)g.col.size();  // >= 2 when connected; 0 for two isolated vertices
    const int k = nnz > 0 ? (int)(rng() % nnz) : 0;
    bool allow_singular = (rng() & 1) != 0;
    int32_t expect = AMG_OK;
    switch (kind) {
      case K_VALID: break;
      case K_COL_RANGE: g.col[k] = (rng() & 1) ? n + (int)(rng() % 3) : -1 - (int)(rng() % 3); expect = AMG_ERR_GRAPH; break;
      case K_SELF_LOOP: g.col[k] = row_of(g, k); expect = AMG_ERR_GRAPH; break;
      case K_UNSORTED: {  // two entries of a row swapped (k's row, else the first row with two)
        int i = row_of(g, k);
        if (g.rp[i + 1] - g.rp[i] < 2)
          for (i = 0; g.rp[i + 1] - g.rp[i] < 2; ++i) {}
        std::swap(g.col[g.rp[i]], g.col[g.rp[i] + 1]);
        expect = AMG_ERR_GRAPH;
        break;
      }
      case K_WEIGHT_NONPOS: g.w[k] = (rng() & 1) ? 0.0 : -0.5; expect = AMG_ERR_GRAPH; break;
      case K_WEIGHT_NAN: g.w[k] = (rng() & 1) ? std::nan("") : std::numeric_limits<double>::infinity(); expect = AMG_ERR_GRAPH; break;
      case K_ASYMMETRIC: g.w[k] += 0.125; expect = AMG_ERR_GRAPH; break;
      case K_D_NEGATIVE: g.d[rng() % n] = -0.5; expect = AMG_ERR_GRAPH; break;
      case K_D_NAN: g.d[rng() % n] = std::nan(""); expect = AMG_ERR_GRAPH; break;
      case K_ROW_PTR_DECREASING: {
        int i = 1 + (int)(rng() % (n - 1));  // an interior entry made smaller than its predecessor
        while (g.rp[i - 1] == 0 && i < n) ++i;
        if (g.rp[i - 1] > 0) g.rp[i] = g.rp[i - 1] - 1;
        else g.rp[0] = 1;  // all earlier rows empty: break the first entry instead
        expect = AMG_ERR_GRAPH;
        break;
      }
      case K_ROW_PTR_START: g.rp[0] = 1; expect = AMG_ERR_GRAPH; break;
      case K_DISCONNECTED: expect = AMG_ERR_DISCONNECTED; break;
      case K_ALL_D_ZERO: std::fill(g.d.begin(), g.d.end(), 0.0); allow_singular = false; expect = AMG_ERR_SINGULAR; break;
      case K_ALL_D_ZERO_ALLOWED: std::fill(g.d.begin(), g.d.end(), 0.0); allow_singular = true; expect = AMG_OK; break;
      default: break;
    }
    std::string msg;
    const int32_t got = amg::validate_graph(n, g.rp.data(), g.col.data(), g.w.data(), g.d.data(), msg, allow_singular);
    if (got != expect) {
      std::printf("FAIL trial %d kind %s n %d: status %d, expected %d (%s)\n", t, kNames[kind], n, got, expect,
                  msg.c_str());
      return 1;
    }
    ++seen[kind];
  }
  // argument errors: no vertices, missing arrays
  {
    std::string msg;
    const int32_t rp[2] = {0, 0};
    const double d[1] = {1.0};
    if (amg::validate_graph(0, rp, nullptr, nullptr, d, msg, false) != AMG_ERR_ARG ||
        amg::validate_graph(1, rp, nullptr, nullptr, nullptr, msg, false) != AMG_ERR_ARG ||
        amg::validate_graph(1, nullptr, nullptr, nullptr, d, msg, false) != AMG_ERR_ARG ||
        amg::validate_graph(1, rp, nullptr, nullptr, d, msg, false) != AMG_OK) {
      std::printf("FAIL argument checks\n");
      return 1;
    }
  }
  for (int i = 0; i < K_COUNT; ++i) std::printf("%s %d\n", kNames[i], seen[i]);
  return 0;
}
