// Shared declarations of the HIP library: device structures of a level and of
// the hierarchy, error handling, and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "amg.h"

namespace amg {

constexpr int kWave = 64;  // CDNA wavefront width
// Largest level the one-workgroup tail program takes (its plain layout is
// kept for levels up to this size).
constexpr int kTailMaxRows = 4096;

struct Status {
  int32_t code = AMG_OK;
  std::string msg;
};

// Any HIP error becomes AMG_ERR_DEVICE (or NOMEM for failed allocations).
#define AMG_HIP(...)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (__VA_ARGS__);                                                      \
    if (e_ != hipSuccess) {                                                             \
      ::amg::set_last_error(std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_));  \
      return e_ == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;                \
    }                                                                                   \
  } while (0)

#define AMG_TRY(...)                  \
  do {                                \
    int32_t s_ = (__VA_ARGS__);       \
    if (s_ != AMG_OK) return s_;      \
  } while (0)

void set_last_error(const std::string& m);

// Device buffer owned by a hierarchy.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Off-diagonal part of a level in CSR (setup form, also kept for export) and
// in sliced ELL (solve form).  The sliced-ELL layout has three knobs, chosen
// per level at setup: the slice height C (rows per slice), the lanes per row
// K, and whether rows are sorted by length inside each 64-row group.  Slot q
// holds row perm[q] (q itself when unsorted); slot q lies in slice q / C at
// position p = q mod C, and entry k of its row sits at
// sell_off[s] + (k / K) * C * K + p * K + (k mod K).  sell_w[s] is the number
// of steps (entries per lane) of slice s.  Padding entries point at the row
// itself with weight 0.
struct Level {
  int32_t n = 0;
  int64_t nnz = 0;
  // CSR (device)
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  double* W = nullptr;
  double* d = nullptr;
  double* D = nullptr;
  // sliced ELL (device)
  int32_t nslices = 0;
  int32_t* sell_off = nullptr;   // nslices + 1
  int32_t* sell_w = nullptr;     // width of each slice
  int32_t* sell_col = nullptr;
  double* sell_val = nullptr;    // FP64 weights
  float* sell_valf = nullptr;    // FP32 weights (mixed precision)
  float* Df = nullptr;           // FP32 diagonal (mixed precision)
  int64_t sell_entries = 0;
  int32_t sell_lc = 6;           // log2 slice height
  int32_t sell_lk = 0;           // log2 lanes per row
  int32_t* sell_perm = nullptr;  // slot -> row (sorted layouts), else null
  // The plain layout (64-row slices, rows in order, one lane per row) of a
  // small level: the layout the one-workgroup tail program runs on, so that
  // the tail does not depend on the layout chosen for the level (the arrays
  // above when that is the plain layout).
  int32_t plain_nslices = 0;
  int64_t plain_entries = 0;
  int32_t* plain_off = nullptr;
  int32_t* plain_w = nullptr;
  int32_t* plain_col = nullptr;
  double* plain_val = nullptr;
  float* plain_valf = nullptr;
  // aggregation into the next level (device), l < L
  int32_t* agg = nullptr;        // n
  int32_t* members = nullptr;    // n: vertices grouped by aggregate, increasing index
  int32_t* member_off = nullptr; // n_{l+1} + 1
  // smoother
  double lambda1 = 0.0;
  double theta = 0.0, eta = 0.0;
  std::vector<double> coef;      // c_k / eta (so that q_m(A) v = sum_k coef_k w_k)
};

struct Hier;

}  // namespace amg
