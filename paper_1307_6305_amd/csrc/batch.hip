// Batched solve: many independent systems (uneven graphs, or several
// right-hand sides on one hierarchy) advance together through flexible CG with
// the k-cycle preconditioner (Sections 3-4 of the paper).
//
// Execution is level-synchronous over the union of the items' cycles: every
// step of the cycle (a Chebyshev step on level l, a residual, a restriction,
// an inner flexible-CG update, ...) is ONE launch that covers that step for
// every item that takes it, with a block -> item map; each item's small
// levels run as that item's recorded LDS-resident tail program, one workgroup
// per item, all items in one launch.  Inner products are per-item fixed-order
// reductions, convergence is decided per item on the device, and converged
// items are frozen (their blocks return at once).  An item's arithmetic never
// depends on which other items share the launches, so its result is the same
// alone and in any mix.  One outer iteration of the whole batch is captured as
// a HIP graph and replayed; the host reads one counter per replay.
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "batch.h"
#include "kernels.h"

namespace amg {
namespace {

enum BatchOpType : int {
  B_CHEB_FIRST = 1,
  B_CHEB_NEXT,
  B_SCALE_ADD,
  B_RESIDUAL,
  B_RESTRICT,
  B_PROLONG,
  B_COARSE,
  B_MULTIDOT,
  B_FCG_P,
  B_SPMV_DOTS,
  B_FCG_XR,
  B_O_RESID,     // r = f - A u (FP64), (r, r) -> rr0; starts the item
  B_O_MULTIDOT,  // (z, q_i), i < j = iter mod restart
  B_O_P,         // p_j = z - sum beta_i p_i
  B_O_SPMV,      // q_j = A p_j (FP64), (p_j, q_j), (p_j, r)
  B_O_XR,        // u += alpha p_j, r -= alpha q_j, (r, r); convergence
  B_O_TRUE,      // true residual (f - A u, f - A u)
  B_O_CONFIRM,   // items whose recursive residual passed: r = f - A u, (r, r)
};

// Rows per tile (= block) of a batched step: one wavefront, so that many
// blocks -- each first fetching its op's descriptor -- are in flight per CU.
// Reductions leave one partial sum per tile; the rows of a tile are added in
// row order whatever the layout (sorting never moves a row across 64-row
// groups).
constexpr int kBatchRows = 64;

struct BatchOp {
  int type;
  int item;
  int n;
  int k;
  int i0, i1, i2, i3;
  int first_block;  // block of this op's tile 0 in its launch
  int blocks;       // tiles of kBatchRows rows
  int part;         // first partial-sum tile of this op (8 doubles per tile)
  int stride;       // blocks between two tiles of this op (1, or the size of its shared-matrix group)
  double f0, f1, f2, f3;
  Mat<double> A64;
  Mat<float> A32;
  Transfer T;
  CoarseView C;
  const void* a;
  const void* b;
  void* c;
  void* d;
  VecPtrs w;
  VecPtrs w2;
  Slots s0, s1;
  double* scal;
  ItemState* st;
};

template <typename MT>
__device__ __forceinline__ const Mat<MT>& op_mat(const BatchOp& op);
template <>
__device__ __forceinline__ const Mat<double>& op_mat<double>(const BatchOp& op) {
  return op.A64;
}
template <>
__device__ __forceinline__ const Mat<float>& op_mat<float>(const BatchOp& op) {
  return op.A32;
}

// Partial sums of the first kn of K values of this block, for op-local tile `tile`.
template <int K>
__device__ __forceinline__ void deposit(double (&v)[K], double* partials, int slot, double* red, int kn = K) {
  block_sum_k<K>(v, kn, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[(size_t)slot * 8 + k] = v[k];
  }
}

// Steps that multiply by a level's matrix: one tile (kBatchRows rows) of one
// op, with K = 2^lk lanes per row (the launch has kBatchRows << lk threads).
// Reductions leave one partial sum per tile, added in row order.
// TYPE: 0 for any matrix step (a switch on the op's type), or the one op type
// of a launch, so that its kernel holds only that step's code (fewer
// registers, more waves per SIMD).
template <typename VT, typename MT, int TYPE = 0>
__device__ __forceinline__ void batch_mat_tile(const BatchOp& op, int tile, double* partials, double* red,
                                               double* stage) {
  const int lk = op.A64.lk;
  const int slot = tile * kBatchRows + (threadIdx.x >> lk);
  const int lane = threadIdx.x & ((1 << lk) - 1);
  const bool slive = threadIdx.x < (kBatchRows << lk) && slot < op.n;
  const bool stage_rows = needs_stage(op.A64);
  switch (TYPE ? TYPE : op.type) {
    case B_CHEB_FIRST: {
      if (!slive) break;
      const Mat<MT>& A = op_mat<MT>(op);
      // w.p[0]: a coarse correction whose prolongation is folded into y
      const VT* e = (const VT*)op.w.p[0];
      const int* agg = e ? op.T.agg : nullptr;
      if (op.i2)
        row_cheb_first<VT, MT, double>(A, slot, lane, (const double*)op.a, (VT*)op.c, (VT*)op.d, op.f0, op.f1, op.f2,
                                       op.f3, op.i0, op.i1, e, agg);
      else
        row_cheb_first<VT, MT, VT>(A, slot, lane, (const VT*)op.a, (VT*)op.c, (VT*)op.d, op.f0, op.f1, op.f2, op.f3,
                                   op.i0, op.i1, e, agg);
      break;
    }
    case B_CHEB_NEXT: {
      if (!slive) break;
      const Mat<MT>& A = op_mat<MT>(op);
      if (op.i2)
        row_cheb_next<VT, MT, double>(A, slot, lane, (const VT*)op.a, (const double*)op.b, (VT*)op.c, (VT*)op.d,
                                      op.f0, op.f1, op.f2, op.i0);
      else
        row_cheb_next<VT, MT, VT>(A, slot, lane, (const VT*)op.a, (const VT*)op.b, (VT*)op.c, (VT*)op.d, op.f0, op.f1,
                                  op.f2, op.i0);
      break;
    }
    case B_RESIDUAL: {
      if (!slive) break;
      const Mat<MT>& A = op_mat<MT>(op);
      const VT* e = (const VT*)op.w.p[0];  // residual after the prolongation of e
      if (e) {
        if (op.i2)
          (void)row_residual_p<VT, MT, double>(A, slot, lane, (const double*)op.a, (const VT*)op.b, e, op.T.agg,
                                               (VT*)op.c);
        else
          (void)row_residual_p<VT, MT, VT>(A, slot, lane, (const VT*)op.a, (const VT*)op.b, e, op.T.agg, (VT*)op.c);
      } else if (op.i2) {
        (void)row_residual<VT, MT, double>(A, slot, lane, (const double*)op.a, (const VT*)op.b, (VT*)op.c);
      } else {
        (void)row_residual<VT, MT, VT>(A, slot, lane, (const VT*)op.a, (const VT*)op.b, (VT*)op.c);
      }
      break;
    }
    case B_SPMV_DOTS: {
      double v[2] = {0.0, 0.0};
      int row = -1;
      if (slive)
        row = row_spmv_dots<VT, MT, VT>(op_mat<MT>(op), slot, lane, (const VT*)op.a, (VT*)op.c, (const VT*)op.b, v);
      if (stage_rows) tile_stage<2, kBatchRows>(v, row >= 0 ? row - tile * kBatchRows : -1, stage);
      deposit<2>(v, partials, op.part + tile, red);
      break;
    }
    case B_O_RESID:
    case B_O_TRUE:
    case B_O_CONFIRM: {
      double v[1] = {0.0};
      int row = -1;
      if (slive) {
        double* s = (double*)op.c;
        row = row_residual<double, double, double>(op.A64, slot, lane, (const double*)op.a, (const double*)op.b, s);
        if (row >= 0) v[0] = s[row] * s[row];
      }
      if (stage_rows) tile_stage<1, kBatchRows>(v, row >= 0 ? row - tile * kBatchRows : -1, stage);
      deposit<1>(v, partials, op.part + tile, red);
      break;
    }
    case B_O_SPMV: {
      const int j = op.st->pos;
      double v[2] = {0.0, 0.0};
      int row = -1;
      if (slive)
        row = row_spmv_dots<double, double, double>(op.A64, slot, lane, (const double*)op.w2.p[j],
                                                    (double*)op.w.p[j], (const double*)op.b, v);
      if (stage_rows) tile_stage<2, kBatchRows>(v, row >= 0 ? row - tile * kBatchRows : -1, stage);
      deposit<2>(v, partials, op.part + tile, red);
      break;
    }
    default:
      break;
  }
}

// Vector steps: row r of the tile in thread r - tile * kBatchRows.
template <typename VT>
__device__ __forceinline__ void batch_vec_tile(const BatchOp& op, int tile, double* partials, double* red) {
  const int r = tile * kBatchRows + threadIdx.x;
  const bool live = r < op.n;
  switch (op.type) {
    case B_SCALE_ADD: {
      if (!live) break;
      VT* y = (VT*)op.d;
      const VT w0 = op.i2 ? (VT)((const double*)op.a)[r] : ((const VT*)op.a)[r];
      VT v = (VT)op.f0 * w0;
      if (op.i0) v += y[r];
      y[r] = v;
      break;
    }
    case B_RESTRICT:
      if (live) row_restrict<VT>(op.T, r, (const VT*)op.a, (VT*)op.c);
      break;
    case B_PROLONG:
      if (live) row_prolong<VT>(op.T, r, (const VT*)op.a, (VT*)op.c);
      break;
    case B_MULTIDOT: {
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.0;
      if (live) {
        const double zr = (double)((const VT*)op.a)[r];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i < op.k) v[i] = zr * (double)((const VT*)op.w.p[i])[r];
      }
      deposit<8>(v, partials, op.part + tile, red, op.k);
      break;
    }
    case B_FCG_P: {
      if (!live) break;
      double acc = (double)((const VT*)op.a)[r];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < op.k) acc -= fcg_beta(op.scal, op.s0.s[i], op.s1.s[i]) * (double)((const VT*)op.w.p[i])[r];
      ((VT*)op.c)[r] = (VT)acc;
      break;
    }
    case B_FCG_XR: {
      if (!live) break;
      const double alpha = fcg_alpha(op.scal, op.i0, op.i1);
      const double pr = (double)((const VT*)op.a)[r];
      VT* x = (VT*)op.c;
      x[r] = (VT)(op.i2 ? alpha * pr : (double)x[r] + alpha * pr);
      if (op.i3) {
        VT* rv = (VT*)op.d;
        rv[r] = (VT)((double)rv[r] - alpha * (double)((const VT*)op.b)[r]);
      }
      break;
    }
    case B_O_MULTIDOT: {
      const int j = op.st->pos;
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.0;
      if (live) {
        const double zr = (double)((const VT*)op.a)[r];
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (i < j) v[i] = zr * ((const double*)op.w.p[i])[r];
      }
      deposit<8>(v, partials, op.part + tile, red, j);
      break;
    }
    case B_O_P: {
      if (!live) break;
      const int j = op.st->pos;
      double acc = (double)((const VT*)op.a)[r];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < j) acc -= fcg_beta(op.scal, S_DOTS + i, S_RHOW + i) * ((const double*)op.w2.p[i])[r];
      ((double*)op.w2.p[j])[r] = acc;
      break;
    }
    case B_O_XR: {
      const int j = op.st->pos;
      double v[1] = {0.0};
      if (live) {
        const double alpha = fcg_alpha(op.scal, S_RHOW + j, S_GAM);
        double* u = (double*)op.c;
        double* rv = (double*)op.d;
        u[r] += alpha * ((const double*)op.w2.p[j])[r];
        const double rn = rv[r] - alpha * ((const double*)op.w.p[j])[r];
        rv[r] = rn;
        v[0] = rn * rn;
      }
      deposit<1>(v, partials, op.part + tile, red);
      break;
    }
    default:
      break;
  }
}

bool is_matrix_step(int type) {
  return type == B_CHEB_FIRST || type == B_CHEB_NEXT || type == B_RESIDUAL || type == B_SPMV_DOTS ||
         type == B_O_RESID || type == B_O_TRUE || type == B_O_SPMV || type == B_O_CONFIRM;
}

// Whether an op runs for an item in the state S: the start and the final
// true residual always; the confirmation only after a pass of the recursive
// test; every other step while the item iterates.
__device__ __forceinline__ bool op_runs(int type, const ItemState& S) {
  if (type == B_O_RESID || type == B_O_TRUE) return true;
  if (type == B_O_CONFIRM) return S.active && S.check;
  return S.active;
}

// One step of the cycle for every item of the launch.  Block b works on tile
// (b - first_block) / stride of op block_op[b].  Matrix and vector steps are separate
// kernels, each with the registers its own code needs.
template <typename VT, typename MT, int TYPE>
__global__ void __launch_bounds__(kBatchRows * 4) k_batch_mat(const BatchOp* __restrict__ ops,
                                                       const int* __restrict__ block_op, double* partials) {
  __shared__ double red[16 * 8];
  __shared__ double stage[2 * kBatchRows];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const BatchOp& op = ops[block_op[b]];
  if (!op_runs(op.type, *op.st)) return;
  batch_mat_tile<VT, MT, TYPE>(op, (b - op.first_block) / op.stride, partials, red, stage);
}

// One tile of a group of G ops that share a matrix (the right-hand sides of one
// hierarchy): the lane loads its row's entries once -- when the slice is at
// most one batch wide -- and applies them to every op of the group in turn,
// each with the arithmetic of the op's own row step (the same bits as alone).
// Wider slices take every op through its usual tile.
template <typename VT, typename MT, int TYPE, int K>
__device__ __forceinline__ void batch_group_tile(const BatchOp* __restrict__ ops, int g0, int G, int tile,
                                                 double* partials, double* red, double* stage) {
  const BatchOp& o0 = ops[g0];
  const int slot = tile * kBatchRows + (threadIdx.x / K);
  const int lane = threadIdx.x % K;
  if (!(threadIdx.x < kBatchRows * K && slot < o0.n)) return;  // these steps do not reduce
  const Mat<MT>& A = op_mat<MT>(o0);
  if (A.width[slot >> A.lc] > OffPre<K, MT>::U) {
    for (int g = 0; g < G; ++g) {
      const BatchOp& op = ops[g0 + g];
      if (op_runs(op.type, *op.st)) batch_mat_tile<VT, MT, TYPE>(op, tile, partials, red, stage);
    }
    return;
  }
  OffPre<K, MT> P;
  P.load(A, slot, lane);
  for (int g = 0; g < G; ++g) {
    const BatchOp& op = ops[g0 + g];
    if (!op_runs(op.type, *op.st)) continue;
    if constexpr (TYPE == B_CHEB_NEXT) {
      if (op.i2)
        row_cheb_next<VT, MT, double, false, OffPre<K, MT>>(A, slot, lane, (const VT*)op.a, (const double*)op.b,
                                                                   (VT*)op.c, (VT*)op.d, op.f0, op.f1, op.f2, op.i0, P);
      else
        row_cheb_next<VT, MT, VT, false, OffPre<K, MT>>(A, slot, lane, (const VT*)op.a, (const VT*)op.b,
                                                               (VT*)op.c, (VT*)op.d, op.f0, op.f1, op.f2, op.i0, P);
    } else if constexpr (TYPE == B_CHEB_FIRST) {
      const VT* e = (const VT*)op.w.p[0];
      const int* agg = e ? op.T.agg : nullptr;
      if (op.i2)
        row_cheb_first<VT, MT, double, OffPre<K, MT>>(A, slot, lane, (const double*)op.a, (VT*)op.c, (VT*)op.d,
                                                            op.f0, op.f1, op.f2, op.f3, op.i0, op.i1, e, agg, P);
      else
        row_cheb_first<VT, MT, VT, OffPre<K, MT>>(A, slot, lane, (const VT*)op.a, (VT*)op.c, (VT*)op.d, op.f0,
                                                        op.f1, op.f2, op.f3, op.i0, op.i1, e, agg, P);
    } else if constexpr (TYPE == B_RESIDUAL) {
      const VT* e = (const VT*)op.w.p[0];
      if (e) {
        if (op.i2)
          (void)row_residual_p<VT, MT, double, OffPre<K, MT>>(A, slot, lane, (const double*)op.a,
                                                                    (const VT*)op.b, e, op.T.agg, (VT*)op.c, P);
        else
          (void)row_residual_p<VT, MT, VT, OffPre<K, MT>>(A, slot, lane, (const VT*)op.a, (const VT*)op.b, e,
                                                                op.T.agg, (VT*)op.c, P);
      } else if (op.i2) {
        (void)row_residual<VT, MT, double, OffPre<K, MT>>(A, slot, lane, (const double*)op.a, (const VT*)op.b,
                                                                (VT*)op.c, P);
      } else {
        (void)row_residual<VT, MT, VT, OffPre<K, MT>>(A, slot, lane, (const VT*)op.a, (const VT*)op.b,
                                                            (VT*)op.c, P);
      }
    }
  }
}

// Grouped matrix steps: block b takes one tile for the group of ops that
// starts at block_op[b] (stride = the group's size, first_block its first
// block).
template <typename VT, typename MT, int TYPE>
__global__ void __launch_bounds__(kBatchRows * 4) k_batch_mat_group(const BatchOp* __restrict__ ops,
                                                             const int* __restrict__ block_op, double* partials) {
  __shared__ double red[16 * 8];
  __shared__ double stage[2 * kBatchRows];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int g0 = block_op[b];
  const BatchOp& o0 = ops[g0];
  const int tile = b - o0.first_block;
  if (o0.A64.lk == 0)
    batch_group_tile<VT, MT, TYPE, 1>(ops, g0, o0.stride, tile, partials, red, stage);
  else if (o0.A64.lk == 1)
    batch_group_tile<VT, MT, TYPE, 2>(ops, g0, o0.stride, tile, partials, red, stage);
  else
    batch_group_tile<VT, MT, TYPE, 4>(ops, g0, o0.stride, tile, partials, red, stage);
}

template <typename VT>
__global__ void __launch_bounds__(kBatchRows) k_batch_vec(const BatchOp* __restrict__ ops, const int* __restrict__ block_op,
                                                   double* partials) {
  __shared__ double red[16 * 8];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const BatchOp& op = ops[block_op[b]];
  if (!op.st->active) return;
  batch_vec_tile<VT>(op, (b - op.first_block) / op.stride, partials, red);
}

// Coarsest solves, one block per item.
template <typename VT>
__global__ void __launch_bounds__(TPB) k_batch_coarse(const BatchOp* __restrict__ ops) {
  __shared__ double sb[1024], sy[1024];
  const BatchOp& op = ops[blockIdx.x];
  if (!op.st->active) return;
  if (op.i2)
    coarse_apply<VT, double>(op.C, (const double*)op.a, (VT*)op.c, sb, sy);
  else
    coarse_apply<VT, VT>(op.C, (const VT*)op.a, (VT*)op.c, sb, sy);
}

// Tail programs, one workgroup per item.
template <typename VT, typename MT>
__global__ void __launch_bounds__(TAIL_THREADS) k_batch_tail(const TailProgram* __restrict__ progs,
                                                             ItemState* const* __restrict__ states) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double red[16 * 8];
  __shared__ double sb[1024], sy[1024];
  if (!states[blockIdx.x]->active) return;
  run_tail<VT, MT>(progs[blockIdx.x], lds, red, sb, sy, true);
}

// Fixed-order sums of each reduction op's partials (one block per op), and
// the per-item bookkeeping of the outer iteration.
__global__ void __launch_bounds__(kFinishThreads) k_batch_finish(const BatchOp* __restrict__ ops,
                                                                 const int* __restrict__ fin, const double* partials,
                                                                 BatchCtl ctl) {
  __shared__ double red[16 * 8];
  const BatchOp& op = ops[fin[blockIdx.x]];
  ItemState& S = *op.st;
  if (!op_runs(op.type, S)) return;
  double acc[8];
  sum_partials<8>(partials + (size_t)op.part * 8, op.blocks, acc, red);
  if (threadIdx.x != 0) return;
  switch (op.type) {
    case B_MULTIDOT:
      for (int i = 0; i < op.k; ++i) op.scal[op.s0.s[i]] = acc[i];
      break;
    case B_SPMV_DOTS:
      op.scal[op.s0.s[0]] = acc[0];
      op.scal[op.s0.s[1]] = acc[1];
      break;
    case B_O_MULTIDOT: {
      const int j = S.pos;
      for (int i = 0; i < j; ++i) op.scal[S_DOTS + i] = acc[i];
      break;
    }
    case B_O_SPMV: {
      const int j = S.pos;
      op.scal[S_RHOW + j] = acc[0];
      op.scal[S_GAM] = acc[1];
      break;
    }
    case B_O_RESID:
      S.rr0 = acc[0];
      S.rr = acc[0];
      S.iter = 0;
      S.pos = 0;
      S.check = 0;
      S.replaced = 0;
      S.status = AMG_OK;
      S.active = acc[0] > 0.0 ? 1 : 0;
      if (S.active) atomicAdd(ctl.nactive, 1);
      break;
    case B_O_TRUE:
      S.rrt = acc[0];
      break;
    case B_O_XR: {
      const int j = S.pos;
      const double rho = op.scal[S_RHOW + j];
      S.iter += 1;
      S.pos = j + 1 == op.i0 ? 0 : j + 1;
      S.rr = acc[0];
      bool stop = false;
      if (!(rho > 0.0) || !isfinite(rho)) {
        S.status = AMG_ERR_BREAKDOWN;
        stop = true;
      } else if (acc[0] <= ctl.tol * ctl.tol * S.rr0) {
        S.check = 1;  // the confirmation step decides on the true residual
      } else if (S.iter >= ctl.max_iter) {
        S.status = AMG_ERR_MAXIT;
        stop = true;
      }
      if (stop) {
        S.active = 0;
        atomicSub(ctl.nactive, 1);
      }
      break;
    }
    case B_O_CONFIRM: {
      // r = f - A u has replaced the recursive residual: stop when it passes,
      // else restart the window from it
      S.check = 0;
      S.rr = acc[0];
      S.rrt = acc[0];
      bool stop = false;
      if (acc[0] <= ctl.tol * ctl.tol * S.rr0) {
        S.status = AMG_OK;
        stop = true;
      } else {
        S.pos = 0;
        S.replaced += 1;
        if (S.iter >= ctl.max_iter) {
          S.status = AMG_ERR_MAXIT;
          stop = true;
        }
      }
      if (stop) {
        S.active = 0;
        atomicSub(ctl.nactive, 1);
      }
      break;
    }
    default:
      break;
  }
}

__global__ void k_batch_reset(int* nactive) { *nactive = 0; }

// ------------------------------------------------------------------ schedule
}  // namespace

// Grouped matrix steps: at most kGroupMax ops per block, on levels of at
// least kGroupMinTiles tiles.
constexpr int kGroupMax = 8;
constexpr int kGroupMinTiles = 1024;

struct Launch {
  int kind;  // 0 vector step, 4 matrix step, 5 grouped matrix step, 1 coarse, 2 tail, 3 finish
  int optype;  // the op type of a step launch
  int op0, nops;
  int map0, nblocks;  // block map slice (step) / finish list slice
  int tail0;          // first tail program (tail)
  size_t lds;         // dynamic LDS (tail)
  int threads;
};

// The schedule's device arrays, packed into one buffer that later builds of
// the same Schedule reuse (it only grows), so that rebuilding a schedule --
// the server does so whenever slots join -- costs no allocation and no free
// (a free synchronizes the whole device).
struct ScheduleDev {
  BatchOp* ops = nullptr;
  int* map = nullptr;
  int* fin = nullptr;
  TailProgram* tails = nullptr;
  ItemState** tail_states = nullptr;
  double* partials = nullptr;
  char* buf = nullptr;
  size_t cap = 0;
  std::vector<char> staging;  // host image of the uploaded arrays
};

namespace {

// Builds the union schedule of the items' cycles.
struct Builder {
  const std::vector<BatchItem>& items;
  bool mixed;
  std::vector<Launch>* out;
  std::vector<BatchOp> ops;
  std::vector<int> map;
  std::vector<int> fin;
  std::vector<TailProgram> tails;
  std::vector<ItemState*> tail_states;
  int max_parts = 0;  // largest partial-sum need over launches (the buffer is reused)

  Builder(const std::vector<BatchItem>& it, bool mx, std::vector<Launch>* o) : items(it), mixed(mx), out(o) {}

  BatchOp blank(int type, int item) const {
    BatchOp o;
    std::memset(&o, 0, sizeof(o));
    o.type = type;
    o.item = item;
    o.st = items[item].st;
    return o;
  }

  const amg_hier* H(int i) const { return items[i].h; }

  void fill_mats(BatchOp& o, int i, int l) const {
    const Level& lv = H(i)->lv[l];
    o.A64 = mat_of<double>(lv);
    if (mixed) o.A32 = mat_of<float>(lv);
  }

  // One step over the given ops (each spanning ceil(n / kBatchRows) tiles): one
  // launch per lanes-per-row value among them, so that every block has the
  // thread count its op's layout uses.
  void step(std::vector<BatchOp> v, bool reduces) {
    if (v.empty()) return;
    int present = 0;
    for (const BatchOp& o : v) present |= 1 << o.A64.lk;
    if ((present & (present - 1)) == 0) {
      step_launch(std::move(v), reduces);
      return;
    }
    for (int lk = 0; lk <= 2; ++lk) {
      std::vector<BatchOp> part;
      for (const BatchOp& o : v)
        if (o.A64.lk == lk) part.push_back(o);
      if (!part.empty()) step_launch(std::move(part), reduces);
    }
  }

  // Matrix steps of items that share a matrix (several right-hand sides on
  // one hierarchy) are grouped and their blocks interleaved tile by tile:
  // consecutive blocks -- on the same XCD, see xcd_remap -- take the same
  // tile for the group's items one after the other, so the tile's matrix
  // entries come from L2 for all but the first.  Each op's arithmetic and its
  // partial sums (slot part + tile) do not depend on the block order.
  void step_launch(std::vector<BatchOp> v, bool reduces) {
    Launch L{};
    L.kind = is_matrix_step(v[0].type) ? 4 : 0;
    L.optype = v[0].type;
    std::vector<int> group_of(v.size(), 0);  // ops of one group are adjacent after this
    if (L.kind == 4) {
      std::vector<BatchOp> sorted;
      std::vector<char> taken(v.size(), 0);
      int g = 0;
      for (size_t q = 0; q < v.size(); ++q) {
        if (taken[q]) continue;
        for (size_t r = q; r < v.size(); ++r)
          if (!taken[r] && v[r].A64.col == v[q].A64.col && v[r].n == v[q].n && v[r].A64.lk == v[q].A64.lk) {
            taken[r] = 1;
            sorted.push_back(v[r]);
            group_of[sorted.size() - 1] = g;
          }
        ++g;
      }
      v.swap(sorted);
    } else {
      for (size_t q = 0; q < v.size(); ++q) group_of[q] = (int)q;
    }
    L.op0 = (int)ops.size();
    L.nops = (int)v.size();
    L.map0 = (int)map.size();
    int parts = 0, blocks = 0;
    // Grouped layout (kind 5): one block per tile and group of at most
    // kGroupMax ops -- for steps that do not reduce, when some group of at
    // least two ops spans kGroupMinTiles tiles (smaller levels keep one block
    // per op and tile: a block's ops run one after the other).
    bool grouped = false;
    if (L.kind == 4 && !reduces &&
        (L.optype == B_CHEB_NEXT || L.optype == B_CHEB_FIRST || L.optype == B_RESIDUAL)) {
      for (size_t q0 = 0; q0 < v.size();) {
        size_t q1 = q0 + 1;
        while (q1 < v.size() && group_of[q1] == group_of[q0]) ++q1;
        if (q1 - q0 >= 2 && nblk(v[q0].n, kBatchRows) >= kGroupMinTiles) grouped = true;
        q0 = q1;
      }
    }
    if (grouped) {
      L.kind = 5;
      for (size_t q0 = 0; q0 < v.size();) {
        size_t q1 = q0 + 1;
        while (q1 < v.size() && group_of[q1] == group_of[q0]) ++q1;
        const int T = nblk(v[q0].n, kBatchRows);
        const int gmax = T >= kGroupMinTiles ? kGroupMax : 1;
        for (size_t a = q0; a < q1; a += gmax) {
          const size_t e = std::min(q1, a + gmax);
          for (size_t q = a; q < e; ++q) {
            BatchOp& o = v[q];
            o.blocks = T;
            o.first_block = blocks;
            o.stride = (int)(e - a);
            o.part = 0;
          }
          for (int t = 0; t < T; ++t) map.push_back(L.op0 + (int)a);
          blocks += T;
        }
        q0 = q1;
      }
    }
    for (size_t q0 = 0; q0 < v.size() && !grouped;) {
      size_t q1 = q0 + 1;
      while (q1 < v.size() && group_of[q1] == group_of[q0]) ++q1;
      const int G = (int)(q1 - q0);
      const int T = nblk(v[q0].n, kBatchRows);
      for (size_t q = q0; q < q1; ++q) {
        BatchOp& o = v[q];
        o.blocks = T;
        o.first_block = blocks + (int)(q - q0);
        o.stride = G;
        o.part = parts;
        if (reduces) parts += o.blocks;
      }
      for (int t = 0; t < T; ++t)
        for (size_t q = q0; q < q1; ++q) map.push_back(L.op0 + (int)q);
      blocks += G * T;
      q0 = q1;
    }
    for (const BatchOp& o : v) ops.push_back(o);
    L.nblocks = blocks;
    L.threads = kBatchRows;
    for (const BatchOp& o : v) L.threads = std::max(L.threads, kBatchRows << o.A64.lk);
    max_parts = std::max(max_parts, parts);
    out->push_back(L);
    if (reduces) {
      Launch F{};
      F.kind = 3;
      F.map0 = (int)fin.size();
      F.nblocks = L.nops;
      for (int q = 0; q < L.nops; ++q) fin.push_back(L.op0 + q);
      out->push_back(F);
    }
  }

  // Vectors are named per item: the level's rhs, sol, Z[k], S, A, B buffers,
  // or the outer r / z.
  enum Src { SRC_OUTER_R, SRC_RHS, SRC_S, SRC_Q0 };
  enum Dst { DST_OUTER_Z, DST_Z };

  const void* src_ptr(int i, int l, Src s) const {
    if (s == SRC_OUTER_R) return H(i)->r;
    if (s == SRC_RHS) return H(i)->ws[l].rhs;
    if (s == SRC_Q0) return H(i)->ws[l].Q[0];
    return H(i)->ws[l].S;
  }
  void* dst_ptr(int i, int l, Dst d, int k) const {
    if (d == DST_OUTER_Z) return H(i)->z;
    return H(i)->ws[l].Z[k];
  }

  // fold: y is x before the prolongation of the level's coarse correction
  void smooth(int l, const std::vector<int>& I, Src src, Dst dst, int k, bool accum, bool fold = false) {
    const int m = H(I[0])->p.degree;
    const bool r64 = (src == SRC_OUTER_R) && mixed;
    if (m == 0) {
      std::vector<BatchOp> v;
      for (int i : I) {
        const Level& lv = H(i)->lv[l];
        BatchOp o = blank(B_SCALE_ADD, i);
        o.n = lv.n;
        o.a = src_ptr(i, l, src);
        o.d = dst_ptr(i, l, dst, k);
        o.f0 = lv.coef[0];
        o.i0 = accum;
        o.i2 = r64;
        v.push_back(o);
      }
      step(v, false);
      return;
    }
    {
      std::vector<BatchOp> v;
      for (int i : I) {
        const Level& lv = H(i)->lv[l];
        BatchOp o = blank(B_CHEB_FIRST, i);
        fill_mats(o, i, l);
        o.n = lv.n;
        o.a = src_ptr(i, l, src);
        o.c = H(i)->ws[l].A;
        o.d = dst_ptr(i, l, dst, k);
        o.f0 = lv.theta;
        o.f1 = 1.0 / lv.eta;
        o.f2 = lv.coef[0];
        o.f3 = lv.coef[1];
        o.i0 = accum;
        o.i1 = m > 1;
        o.i2 = r64;
        if (fold) {
          o.w.p[0] = H(i)->ws[l + 1].sol;
          o.T = transfer_of(H(i), l);
        }
        v.push_back(o);
      }
      step(v, false);
    }
    for (int s = 1; s < m; ++s) {
      std::vector<BatchOp> v;
      for (int i : I) {
        const Level& lv = H(i)->lv[l];
        const auto& W = H(i)->ws[l];
        // buffers: w_1 in A; w_2 in B; w_{k+1} overwrites w_{k-1}
        const void* cur = (s % 2 == 1) ? W.A : W.B;
        const void* prev = (s == 1) ? src_ptr(i, l, src) : ((s % 2 == 1) ? W.B : W.A);
        void* next = (s % 2 == 1) ? W.B : W.A;
        BatchOp o = blank(B_CHEB_NEXT, i);
        fill_mats(o, i, l);
        o.n = lv.n;
        o.a = cur;
        o.b = prev;
        o.c = next;
        o.d = dst_ptr(i, l, dst, k);
        o.f0 = lv.theta;
        o.f1 = 2.0 / lv.eta;
        o.f2 = lv.coef[s + 1];
        o.i0 = (s + 1 < m);
        o.i2 = (s == 1) && r64;
        v.push_back(o);
      }
      step(v, false);
    }
  }

  // s = src - A dst; with fold, s = src - A (dst + P e) for the level's
  // coarse correction e (the prolongation itself is left to smooth())
  void residual(int l, const std::vector<int>& I, Src src, Dst dst, int k, bool fold = false) {
    std::vector<BatchOp> v;
    for (int i : I) {
      BatchOp o = blank(B_RESIDUAL, i);
      fill_mats(o, i, l);
      o.n = H(i)->lv[l].n;
      o.a = src_ptr(i, l, src);
      o.b = dst_ptr(i, l, dst, k);
      o.c = H(i)->ws[l].S;
      o.i2 = (src == SRC_OUTER_R) && mixed;
      if (fold) {
        o.w.p[0] = H(i)->ws[l + 1].sol;
        o.T = transfer_of(H(i), l);
      }
      v.push_back(o);
    }
    step(v, false);
  }

  void restrict_(int l, const std::vector<int>& I) {
    std::vector<BatchOp> v;
    for (int i : I) {
      BatchOp o = blank(B_RESTRICT, i);
      o.T = transfer_of(H(i), l);
      o.n = o.T.nc;
      o.a = H(i)->ws[l].S;
      o.c = H(i)->ws[l + 1].rhs;
      v.push_back(o);
    }
    step(v, false);
  }

  void prolong(int l, const std::vector<int>& I, Dst dst, int k) {
    std::vector<BatchOp> v;
    for (int i : I) {
      BatchOp o = blank(B_PROLONG, i);
      o.T = transfer_of(H(i), l);
      o.n = o.T.n;
      o.a = H(i)->ws[l + 1].sol;
      o.c = dst_ptr(i, l, dst, k);
      v.push_back(o);
    }
    step(v, false);
  }

  void coarse_launch(const std::vector<BatchOp>& v) {
    if (v.empty()) return;
    Launch L{};
    L.kind = 1;
    L.op0 = (int)ops.size();
    L.nops = (int)v.size();
    ops.insert(ops.end(), v.begin(), v.end());
    out->push_back(L);
  }

  void coarse(const std::vector<int>& I) {
    std::vector<BatchOp> v;
    for (int i : I) {
      const amg_hier* h = H(i);
      BatchOp o = blank(B_COARSE, i);
      o.C = CoarseView{h->nL, h->chol_inv, h->chol_invT};
      o.a = h->ws[h->L].rhs;
      o.c = h->ws[h->L].sol;
      v.push_back(o);
    }
    coarse_launch(v);
  }

  void tail(const std::vector<int>& I) {
    if (I.empty()) return;
    Launch L{};
    L.kind = 2;
    L.tail0 = (int)tails.size();
    L.nops = (int)I.size();
    L.lds = 0;
    L.threads = 64;
    for (int i : I) {
      const amg_hier* h = H(i);
      tails.push_back(*static_cast<const TailProgram*>(h->tail_prog));
      tail_states.push_back(items[i].st);
      L.lds = std::max(L.lds, h->tail_lds_bytes);
      L.threads = std::max(L.threads, h->tail_threads);
    }
    out->push_back(L);
  }

  // x = Kcycle(l, r) for the items I (all with l < L_i)
  void kcycle(int l, const std::vector<int>& I, Src src, Dst dst, int k) {
    std::vector<int> C, T, R;
    smooth(l, I, src, dst, k, false);
    residual(l, I, src, dst, k);
    restrict_(l, I);
    for (int i : I) {
      const amg_hier* h = H(i);
      if (l + 1 == h->L) C.push_back(i);
      else if (h->tail_level == l + 1) T.push_back(i);
      else R.push_back(i);
    }
    coarse(C);
    tail(T);
    if (!R.empty()) {
      if (H(I[0])->p.cycle == AMG_CYCLE_AMLI)
        amli(l + 1, R);
      else
        inner(l + 1, R);
    }
    if (H(I[0])->p.degree > 0) {
      // the prolongation folded into the residual and the first smoothing step
      residual(l, I, src, dst, k, true);
      smooth(l, I, SRC_S, dst, k, true, true);
      return;
    }
    prolong(l, I, dst, k);
    residual(l, I, src, dst, k);
    smooth(l, I, SRC_S, dst, k, true);
  }

  // The stationary AMLI correction on level l for the items I: sol = g0 y0 +
  // g1 y1 with y0 = B rhs, y1 = B (A y0), the same steps as the single-system
  // solve (the product's inner products go to a dummy slot).
  void amli(int l, const std::vector<int>& I) {
    kcycle(l, I, SRC_RHS, DST_Z, 0);
    {
      std::vector<BatchOp> v;
      for (int i : I) {
        const auto& W = H(i)->ws[l];
        BatchOp o = blank(B_SPMV_DOTS, i);
        fill_mats(o, i, l);
        o.n = H(i)->lv[l].n;
        o.a = W.Z[0];
        o.b = W.Z[0];
        o.c = W.Q[0];
        o.scal = H(i)->scal;
        for (int q = 0; q < 8; ++q) o.s0.s[q] = S_DUMMY;
        v.push_back(o);
      }
      step(v, true);
    }
    kcycle(l, I, SRC_Q0, DST_Z, 1);
    for (int t = 0; t < 2; ++t) {
      std::vector<BatchOp> v;
      for (int i : I) {
        const auto& W = H(i)->ws[l];
        BatchOp o = blank(B_SCALE_ADD, i);
        o.n = H(i)->lv[l].n;
        o.a = W.Z[t];
        o.d = W.sol;
        o.f0 = t == 0 ? H(i)->amli_g0[l] : H(i)->amli_g1[l];
        o.i0 = t;
        v.push_back(o);
      }
      step(v, false);
    }
  }

  // nu flexible-CG steps from zero on level l for the items I
  void inner(int l, const std::vector<int>& I) {
    const int nu = H(I[0])->p.inner_steps;
    const int base = lbase(l);
    for (int k = 0; k < nu; ++k) {
      kcycle(l, I, SRC_RHS, DST_Z, k);
      if (k > 0) {
        std::vector<BatchOp> v, w;
        for (int i : I) {
          const auto& W = H(i)->ws[l];
          BatchOp o = blank(B_MULTIDOT, i);
          o.n = H(i)->lv[l].n;
          o.k = k;
          o.a = W.Z[k];
          for (int q = 0; q < k; ++q) o.w.p[q] = W.Q[q];
          o.scal = H(i)->scal;
          for (int q = 0; q < 8; ++q) o.s0.s[q] = q < k ? base + 16 + q : S_DUMMY;
          v.push_back(o);
          BatchOp p = blank(B_FCG_P, i);
          p.n = o.n;
          p.k = k;
          p.a = W.Z[k];
          p.c = W.Z[k];
          for (int q = 0; q < k; ++q) p.w.p[q] = W.Z[q];
          p.scal = H(i)->scal;
          for (int q = 0; q < 8; ++q) {
            p.s0.s[q] = q < k ? base + 16 + q : S_DUMMY;
            p.s1.s[q] = q < k ? base + q : S_DUMMY;
          }
          w.push_back(p);
        }
        step(v, true);
        step(w, false);
      }
      std::vector<BatchOp> v, w;
      for (int i : I) {
        const auto& W = H(i)->ws[l];
        BatchOp o = blank(B_SPMV_DOTS, i);
        fill_mats(o, i, l);
        o.n = H(i)->lv[l].n;
        o.a = W.Z[k];
        o.b = W.rhs;
        o.c = W.Q[k];
        o.scal = H(i)->scal;
        for (int q = 0; q < 8; ++q) o.s0.s[q] = S_DUMMY;
        o.s0.s[0] = base + k;
        o.s0.s[1] = base + 8 + k;
        v.push_back(o);
        BatchOp x = blank(B_FCG_XR, i);
        x.n = o.n;
        x.a = W.Z[k];
        x.b = W.Q[k];
        x.c = W.sol;
        x.d = W.rhs;
        x.i0 = base + k;
        x.i1 = base + 8 + k;
        x.i2 = (k == 0);
        x.i3 = (k + 1 < nu);
        x.scal = H(i)->scal;
        w.push_back(x);
      }
      step(v, true);
      step(w, false);
    }
  }

  void outer_residual(int type, bool into_r) {
    std::vector<BatchOp> v;
    for (int i = 0; i < (int)items.size(); ++i) {
      BatchOp o = blank(type, i);
      fill_mats(o, i, 0);
      o.n = H(i)->lv[0].n;
      o.a = items[i].f;
      o.b = items[i].u;
      o.c = into_r ? (void*)H(i)->r : (void*)H(i)->tmp;
      v.push_back(o);
    }
    step(v, true);
  }

  void outer_iteration() {
    std::vector<int> all;
    std::vector<BatchOp> one_level;
    for (int i = 0; i < (int)items.size(); ++i) {
      const amg_hier* h = H(i);
      if (h->L > 0) {
        all.push_back(i);
        continue;
      }
      // one-level item: the preconditioner is the coarsest solve itself
      BatchOp o = blank(B_COARSE, i);
      o.C = CoarseView{h->nL, h->chol_inv, h->chol_invT};
      o.a = h->r;
      o.c = h->z;
      o.i2 = mixed;
      one_level.push_back(o);
    }
    coarse_launch(one_level);
    if (!all.empty()) kcycle(0, all, SRC_OUTER_R, DST_OUTER_Z, 0);
    std::vector<BatchOp> md, pp, sp, xr;
    for (int i = 0; i < (int)items.size(); ++i) {
      const amg_hier* h = H(i);
      const int R = h->p.restart;
      BatchOp o = blank(B_O_MULTIDOT, i);
      o.n = h->lv[0].n;
      o.i0 = R;
      o.a = h->z;
      for (int q = 0; q < R; ++q) {
        o.w.p[q] = h->Qo[q];
        o.w2.p[q] = h->P[q];
      }
      o.scal = h->scal;
      md.push_back(o);
      BatchOp p = o;
      p.type = B_O_P;
      pp.push_back(p);
      BatchOp sv = o;
      sv.type = B_O_SPMV;
      fill_mats(sv, i, 0);
      sv.b = h->r;
      sp.push_back(sv);
      BatchOp x = o;
      x.type = B_O_XR;
      x.c = items[i].u;
      x.d = h->r;
      xr.push_back(x);
    }
    step(md, true);
    step(pp, false);
    step(sp, true);
    step(xr, true);
    outer_residual(B_O_CONFIRM, true);
  }
};

template <typename VT, typename MT>
int32_t run_impl(const Schedule* S, const BatchCtl& ctl, hipStream_t s) {
  const ScheduleDev* D = S->dev;
  for (const Launch& L : *S->launches) {
    switch (L.kind) {
      case 0:
        hipLaunchKernelGGL((k_batch_vec<VT>), dim3(L.nblocks), dim3(kBatchRows), 0, s, D->ops, D->map + L.map0,
                           D->partials);
        break;
      case 4:
        // the Chebyshev steps and residuals (most of a cycle's matrix passes)
        // get kernels of their own
        if (L.optype == B_CHEB_NEXT)
          hipLaunchKernelGGL((k_batch_mat<VT, MT, B_CHEB_NEXT>), dim3(L.nblocks), dim3(L.threads), 0, s, D->ops,
                             D->map + L.map0, D->partials);
        else if (L.optype == B_CHEB_FIRST)
          hipLaunchKernelGGL((k_batch_mat<VT, MT, B_CHEB_FIRST>), dim3(L.nblocks), dim3(L.threads), 0, s, D->ops,
                             D->map + L.map0, D->partials);
        else if (L.optype == B_RESIDUAL)
          hipLaunchKernelGGL((k_batch_mat<VT, MT, B_RESIDUAL>), dim3(L.nblocks), dim3(L.threads), 0, s, D->ops,
                             D->map + L.map0, D->partials);
        else
          hipLaunchKernelGGL((k_batch_mat<VT, MT, 0>), dim3(L.nblocks), dim3(L.threads), 0, s, D->ops,
                             D->map + L.map0, D->partials);
        break;
      case 5:
        if (L.optype == B_CHEB_NEXT)
          hipLaunchKernelGGL((k_batch_mat_group<VT, MT, B_CHEB_NEXT>), dim3(L.nblocks), dim3(L.threads), 0, s,
                             D->ops, D->map + L.map0, D->partials);
        else if (L.optype == B_CHEB_FIRST)
          hipLaunchKernelGGL((k_batch_mat_group<VT, MT, B_CHEB_FIRST>), dim3(L.nblocks), dim3(L.threads), 0, s,
                             D->ops, D->map + L.map0, D->partials);
        else
          hipLaunchKernelGGL((k_batch_mat_group<VT, MT, B_RESIDUAL>), dim3(L.nblocks), dim3(L.threads), 0, s,
                             D->ops, D->map + L.map0, D->partials);
        break;
      case 1:
        hipLaunchKernelGGL((k_batch_coarse<VT>), dim3(L.nops), dim3(TPB), 0, s, D->ops + L.op0);
        break;
      case 2:
        hipLaunchKernelGGL((k_batch_tail<VT, MT>), dim3(L.nops), dim3(L.threads), L.lds, s, D->tails + L.tail0,
                           D->tail_states + L.tail0);
        break;
      case 3:
        hipLaunchKernelGGL(k_batch_finish, dim3(L.nblocks), dim3(kFinishThreads), 0, s, D->ops, D->fin + L.map0,
                           D->partials, ctl);
        break;
    }
    AMG_HIP(hipGetLastError());
  }
  return AMG_OK;
}

// Byte offset of the next array in the packed buffer (256-byte aligned).
inline size_t pack_next(size_t off) { return (off + 255) & ~size_t(255); }

}  // namespace

int32_t batch_compatible(const std::vector<amg_hier*>& hs) {
  if (hs.empty()) {
    set_last_error("empty batch");
    return AMG_ERR_ARG;
  }
  const amg_params& p0 = hs[0]->p;
  for (size_t i = 0; i < hs.size(); ++i) {
    const amg_hier* h = hs[i];
    if (h->p.cycle == AMG_CYCLE_AMLI && (int)h->amli_g0.size() < h->L) {
      set_last_error("AMLI coefficients missing");
      return AMG_ERR_ARG;
    }
    if (h->p.stop != AMG_STOP_RESIDUAL) {
      set_last_error("the batched form uses the residual stopping test (AMG_STOP_RESIDUAL) only");
      return AMG_ERR_ARG;
    }
    if (h->mixed != hs[0]->mixed || h->p.degree != p0.degree || h->p.inner_steps != p0.inner_steps ||
        h->p.restart != p0.restart || h->p.cycle != p0.cycle) {
      set_last_error("batched items must share precision, degree, inner steps, restart and cycle");
      return AMG_ERR_ARG;
    }
    if (!h->chol_inv) {
      set_last_error("batched items need a coarsest level of at most 1024 rows");
      return AMG_ERR_ARG;
    }
  }
  return AMG_OK;
}

int32_t schedule_build(Schedule* S, SchedKind kind, const std::vector<BatchItem>& items, hipStream_t s) {
  S->kind = kind;
  S->mixed = items.empty() ? false : items[0].h->mixed;
  delete S->launches;
  S->launches = new std::vector<Launch>();
  if (!S->dev) S->dev = new ScheduleDev();
  if (items.empty()) return AMG_OK;
  Builder bd(items, S->mixed, S->launches);
  if (kind == SCHED_INIT) bd.outer_residual(B_O_RESID, true);
  else if (kind == SCHED_FINAL) bd.outer_residual(B_O_TRUE, false);
  else bd.outer_iteration();
  ScheduleDev* D = S->dev;
  // layout of the packed buffer: ops, map, fin, tails, tail states, partials
  size_t off = 0;
  const size_t o_ops = off;
  off = pack_next(off + sizeof(BatchOp) * bd.ops.size());
  const size_t o_map = off;
  off = pack_next(off + sizeof(int) * bd.map.size());
  const size_t o_fin = off;
  off = pack_next(off + sizeof(int) * bd.fin.size());
  const size_t o_tails = off;
  off = pack_next(off + sizeof(TailProgram) * bd.tails.size());
  const size_t o_ts = off;
  off = pack_next(off + sizeof(ItemState*) * bd.tail_states.size());
  const size_t upload_bytes = off;
  const size_t o_part = off;
  off = pack_next(off + (size_t)std::max(1, bd.max_parts) * 8 * sizeof(double));
  if (off > D->cap) {
    // grow (with room for later, larger batches); the old buffer may still
    // be read by work queued on the stream
    if (D->buf) {
      AMG_HIP(hipStreamSynchronize(s));
      (void)hipFree(D->buf);
      D->buf = nullptr;
      D->cap = 0;
    }
    const size_t want = off + off / 2;
    hipError_t e = hipMalloc(&D->buf, want);
    if (e != hipSuccess) {
      D->buf = nullptr;
      set_last_error(std::string("hipMalloc (batch schedule): ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;
    }
    D->cap = want;
    S->bytes = want;
  }
  D->ops = reinterpret_cast<BatchOp*>(D->buf + o_ops);
  D->map = reinterpret_cast<int*>(D->buf + o_map);
  D->fin = reinterpret_cast<int*>(D->buf + o_fin);
  D->tails = reinterpret_cast<TailProgram*>(D->buf + o_tails);
  D->tail_states = reinterpret_cast<ItemState**>(D->buf + o_ts);
  D->partials = reinterpret_cast<double*>(D->buf + o_part);
  // the previous upload may still be in flight from the staging image
  AMG_HIP(hipStreamSynchronize(s));
  D->staging.assign(upload_bytes, 0);
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (bytes) std::memcpy(D->staging.data() + o, src, bytes);
  };
  put(o_ops, bd.ops.data(), sizeof(BatchOp) * bd.ops.size());
  put(o_map, bd.map.data(), sizeof(int) * bd.map.size());
  put(o_fin, bd.fin.data(), sizeof(int) * bd.fin.size());
  put(o_tails, bd.tails.data(), sizeof(TailProgram) * bd.tails.size());
  put(o_ts, bd.tail_states.data(), sizeof(ItemState*) * bd.tail_states.size());
  AMG_HIP(hipMemcpyAsync(D->buf, D->staging.data(), upload_bytes, hipMemcpyHostToDevice, s));
  size_t max_lds = 0;
  for (const auto& L : *S->launches)
    if (L.kind == 2) max_lds = std::max(max_lds, L.lds);
  if (max_lds) {
    const void* fn = S->mixed ? (const void*)k_batch_tail<float, float> : (const void*)k_batch_tail<double, double>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
  }
  return AMG_OK;
}

int32_t schedule_run(const Schedule* S, const BatchCtl& ctl, hipStream_t s) {
  if (!S->launches || S->launches->empty()) return AMG_OK;
  return S->mixed ? run_impl<float, float>(S, ctl, s) : run_impl<double, double>(S, ctl, s);
}

void schedule_free(Schedule* S) {
  if (S->dev) {
    if (S->dev->buf) (void)hipFree(S->dev->buf);
    delete S->dev;
    S->dev = nullptr;
  }
  delete S->launches;
  S->launches = nullptr;
  S->bytes = 0;
}

namespace {

__global__ void k_reset_count(int* c) { *c = 0; }

// State of the batched entry point: the items of the last call, their
// workspaces and states, and the three phase schedules (the iteration replayed
// as a graph).  Reused while the same (h, f, u) are passed.
struct Batch {
  std::vector<void*> key;
  std::vector<amg_hier*> clones;  // workspaces for repeated hierarchies
  std::vector<BatchItem> items;
  ItemState* d_state = nullptr;
  int* d_nactive = nullptr;
  int* h_nactive = nullptr;
  Schedule init, iter, fini;
  hipGraphExec_t g_iter = nullptr;
  hipStream_t gs = nullptr;
  double tol = 1e-8;
  int max_iter = 200;
  ~Batch() {
    (void)hipDeviceSynchronize();
    if (g_iter) (void)hipGraphExecDestroy(g_iter);
    if (gs) (void)hipStreamDestroy(gs);
    schedule_free(&init);
    schedule_free(&iter);
    schedule_free(&fini);
    if (d_state) (void)hipFree(d_state);
    if (d_nactive) (void)hipFree(d_nactive);
    if (h_nactive) (void)hipHostFree(h_nactive);
    for (amg_hier* c : clones) free_clone(c);
  }
  BatchCtl ctl() const { return BatchCtl{tol, max_iter, 0, d_nactive}; }
};

std::mutex g_batch_mu;
std::unique_ptr<Batch> g_batch;  // the most recent batch (its schedule is reused)

using clk = std::chrono::steady_clock;

int32_t make_batch(int nb, amg_hier* const* hs, const double* const* f, double* const* u, hipStream_t s,
                   std::unique_ptr<Batch>* out) {
  auto B = std::make_unique<Batch>();
  std::vector<amg_hier*> hv(hs, hs + nb);
  AMG_TRY(batch_compatible(hv));
  for (int i = 0; i < nb; ++i) {
    if (hs[i]->p.tol != hs[0]->p.tol || hs[i]->p.max_iter != hs[0]->p.max_iter) {
      set_last_error("batched items must share tol and max_iter");
      return AMG_ERR_ARG;
    }
  }
  B->tol = hs[0]->p.tol;
  B->max_iter = hs[0]->p.max_iter;
  AMG_HIP(hipMalloc(&B->d_state, sizeof(ItemState) * nb));
  AMG_HIP(hipMalloc(&B->d_nactive, sizeof(int)));
  AMG_HIP(hipHostMalloc((void**)&B->h_nactive, sizeof(int), hipHostMallocDefault));
  std::map<const amg_hier*, int> seen;
  for (int i = 0; i < nb; ++i) {
    amg_hier* use = hs[i];
    if (seen.count(hs[i])) {  // another right-hand side on the same hierarchy: its own workspace
      amg_hier* c = nullptr;
      AMG_TRY(make_clone(hs[i], &c, s));
      B->clones.push_back(c);
      use = c;
    }
    seen[hs[i]] = 1;
    B->items.push_back(BatchItem{use, f[i], u[i], B->d_state + i});
  }
  AMG_TRY(schedule_build(&B->init, SCHED_INIT, B->items, s));
  AMG_TRY(schedule_build(&B->iter, SCHED_ITER, B->items, s));
  AMG_TRY(schedule_build(&B->fini, SCHED_FINAL, B->items, s));
  // one outer iteration of the whole batch as a graph, with the count of
  // items still iterating copied to pinned host memory at its end
  AMG_HIP(hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  AMG_HIP(hipStreamBeginCapture(B->gs, hipStreamCaptureModeThreadLocal));
  int32_t st = schedule_run(&B->iter, B->ctl(), B->gs);
  if (st == AMG_OK) {
    hipError_t e = hipMemcpyAsync(B->h_nactive, B->d_nactive, sizeof(int), hipMemcpyDeviceToHost, B->gs);
    if (e != hipSuccess) st = AMG_ERR_DEVICE;
  }
  hipError_t e = hipStreamEndCapture(B->gs, &g);
  if (st != AMG_OK) return st;
  AMG_HIP(e);
  e = hipGraphInstantiate(&B->g_iter, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  AMG_HIP(e);
  *out = std::move(B);
  return AMG_OK;
}

}  // namespace

void drop_batches_using(const amg_hier* h) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (!g_batch) return;
  for (const auto& it : g_batch->items)
    if (it.h == h || it.h->parent == h) {
      g_batch.reset();
      return;
    }
}

int32_t solve_batch(int nb, amg_hier* const* hs, const double* const* f, double* const* u, hipStream_t s,
                    amg_info* infos) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto t0 = clk::now();
  std::vector<void*> key;
  for (int i = 0; i < nb; ++i) {
    key.push_back(hs[i]);
    key.push_back((void*)f[i]);
    key.push_back(u[i]);
  }
  if (!g_batch || g_batch->key != key) {
    g_batch.reset();
    std::unique_ptr<Batch> B;
    AMG_TRY(make_batch(nb, hs, f, u, s, &B));
    B->key = key;
    g_batch = std::move(B);
  }
  Batch* B = g_batch.get();
  hipLaunchKernelGGL(k_reset_count, dim3(1), dim3(1), 0, s, B->d_nactive);
  AMG_TRY(schedule_run(&B->init, B->ctl(), s));
  AMG_HIP(hipMemcpyAsync(B->h_nactive, B->d_nactive, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int active = *B->h_nactive;
  int launched = 0;
  while (active > 0 && launched < B->max_iter) {
    AMG_HIP(hipGraphLaunch(B->g_iter, s));
    AMG_HIP(hipStreamSynchronize(s));
    ++launched;
    active = *B->h_nactive;
  }
  AMG_TRY(schedule_run(&B->fini, B->ctl(), s));
  std::vector<ItemState> hst(nb);
  AMG_HIP(hipMemcpyAsync(hst.data(), B->d_state, nb * sizeof(ItemState), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  int32_t worst = AMG_OK;
  for (int i = 0; i < nb; ++i) {
    const ItemState& S = hst[i];
    const double rho0 = std::sqrt(S.rr0);
    if (infos) {
      infos[i].status = S.status;
      infos[i].iters = S.iter;
      infos[i].rel_res = rho0 > 0 ? std::sqrt(S.rr) / rho0 : 0.0;
      infos[i].rel_res_true = rho0 > 0 ? std::sqrt(S.rrt) / rho0 : 0.0;
      infos[i].solve_ms = ms;
      infos[i].test_iter = S.iter;
      infos[i].replacements = S.replaced;
    }
    if (S.status != AMG_OK && worst == AMG_OK) worst = S.status;
  }
  return worst;
}

}  // namespace amg
