// Internal interface of the batched executor (batch.hip), used by the batched
// solve entry point and by the server (serve.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "hier.h"

namespace amg {

// Per-item solve state, in device memory, owned by whoever owns the item.
struct ItemState {
  int active;  // 1 while the item iterates
  int iter;    // completed outer iterations
  int status;  // AMG_OK, AMG_ERR_MAXIT or AMG_ERR_BREAKDOWN
  int pos;     // window position of the next outer iteration
  int check;   // 1: the recursive residual passed; the true one decides
  int replaced;  // recursive residuals replaced by the true one
  double rr0, rr, rrt;
};

// One system of a batch: the hierarchy whose workspace it uses (the
// hierarchy itself or a workspace clone), its right-hand side and solution
// (device), and its device state.
struct BatchItem {
  amg_hier* h;
  const double* f;
  double* u;
  ItemState* st;
};

struct Launch;
struct ScheduleDev;

// The launches of one phase of the batched solve over a fixed set of items.
enum SchedKind { SCHED_INIT = 0, SCHED_ITER = 1, SCHED_FINAL = 2 };

struct Schedule {
  SchedKind kind = SCHED_ITER;
  bool mixed = false;
  std::vector<Launch>* launches = nullptr;
  ScheduleDev* dev = nullptr;
  size_t bytes = 0;  // device bytes held
};

struct BatchCtl {
  double tol;
  int max_iter;
  int pad;
  int* nactive;  // device counter of items still iterating
};

int32_t schedule_build(Schedule* S, SchedKind kind, const std::vector<BatchItem>& items, hipStream_t s);
int32_t schedule_run(const Schedule* S, const BatchCtl& ctl, hipStream_t s);
void schedule_free(Schedule* S);

// Checks that the items can share launches (same precision, degree, inner
// steps, restart; coarsest level with an inverted factor).
int32_t batch_compatible(const std::vector<amg_hier*>& hs);

}  // namespace amg
