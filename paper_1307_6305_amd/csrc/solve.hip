// Solve phase on the device: flexible CG preconditioned by the nonlinear AMLI
// cycle (k-cycle) with the best-uniform-approximation polynomial smoother
// (Sections 3 and 4 of the paper).
//
// Per-row device functions (one row per lane over sliced ELL, slice height 64
// = one wavefront) implement each step once; two executors use them:
//   * device-wide kernels, one launch per step, for the large levels;
//   * k_tail, a one-workgroup interpreter that runs a recorded op program --
//     the whole inner solve of a small level and everything below it -- with
//     workgroup barriers between the steps, so that the W-cycle's many visits
//     of the small levels cost no kernel launches.
// Steps:
//   cheb_first / cheb_next  one Chebyshev three-term step of q_m(A): SpMV,
//                           recurrence and y += c_k w_k in one pass
//   residual                s = r - A x
//   restrict                b = P^T s, a segmented sum over each aggregate's
//                           member list (P is never stored)
//   prolong                 x += P e, a gather of the aggregate value
//   coarse                  coarsest solve with the inverted Cholesky factor
//   multidot, fcg_p,        flexible-CG steps; inner products are
//   spmv_dots, fcg_xr       deterministic reductions in FP64
//
// Scalars never leave the device inside an iteration; the host reads two
// numbers per outer iteration for the stopping test.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "kernels.h"

namespace amg {
namespace {

// ------------------------------------------------------------------ device-wide kernels
// Row-parallel kernels: one block per tile of TPB rows (XCD-aware order),
// K = 2^lk lanes per row, so blockDim = TPB << lk.
constexpr int kMaxRowThreads = TPB * 4;
// Levels below this many rows fold the prolongation into the next steps.
constexpr int kFoldProlongRows = 1 << 18;

// Outer iterations: the pinned host slots of the stopping test (a pair per
// restart-window position from this index on), and the margin above the
// tolerance of the predicted ratio from which the next iteration is queued
// before the test is read.
constexpr int kPubBase = 8;
constexpr double kAheadFactor = 4.0;

struct SlotLane {
  int tile, slot, lane;
};

template <typename MT>
__device__ __forceinline__ SlotLane slot_of(const Mat<MT>& A) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int slot = tile * TPB + (threadIdx.x >> A.lk);
  return SlotLane{tile, slot < A.n ? slot : -1, (int)threadIdx.x & ((1 << A.lk) - 1)};
}

template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_first(Mat<MT> A, const RT* __restrict__ w0, VT* w1, VT* y,
                                                               double theta, double inv_eta, double c0, double c1,
                                                               int accum, int store, const VT* __restrict__ e,
                                                               const int* __restrict__ agg) {
  const SlotLane q = slot_of(A);
  if (q.slot >= 0)
    row_cheb_first<VT, MT, RT>(A, q.slot, q.lane, w0, w1, y, theta, inv_eta, c0, c1, accum, store, e, agg);
}

// STORE: w_{k+1} is written (every step but the last).  KIND: kStepCoarse
// (levels that stay in the caches), kStepFine (the finest level, when it has
// at least kStreamRows rows: the row's own operands are streamed, see
// row_cheb_next), kStepFineTimed and kStepSmallTimed (the code of kStepFine
// and of kStepCoarse in separate instances for the rotating-copies timing of
// a large or a small finest level, so that profiles report them on their
// own).
constexpr int kStepCoarse = 0, kStepFine = 1, kStepFineTimed = 2, kStepSmallTimed = 3;
constexpr int kStreamRows = 1 << 18;
template <typename VT, typename MT, typename PT, bool STORE, int KIND>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_next(Mat<MT> A, const VT* __restrict__ wk, const PT* wprev,
                                                              VT* wnext, VT* y, double theta, double two_inv_eta,
                                                              double ck) {
  const SlotLane q = slot_of(A);
  if (q.slot >= 0)
    row_cheb_next<VT, MT, PT, KIND == kStepFine || KIND == kStepFineTimed>(A, q.slot, q.lane, wk, wprev, wnext, y,
                                                                                theta, two_inv_eta, ck, STORE);
}

// The last Chebyshev step of a smoothing (w_{k+1} not stored) fused with the
// inner product (y, q) of its result with a vector: the sums k_multidot forms
// -- each tile's rows in row order (staged when the layout permutes or splits
// rows), the tile's partial in the slot of its tile index -- so the same bits,
// one launch fewer.
template <typename VT, typename MT, typename PT>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_next_dot(Mat<MT> A, const VT* __restrict__ wk, const PT* wprev,
                                                                  VT* y, double theta, double two_inv_eta, double ck,
                                                                  const VT* __restrict__ q, Red red) {
  __shared__ double stage[TPB];
  const SlotLane sl = slot_of(A);
  double v[1] = {0.0};
  int r = -1;
  if (sl.slot >= 0) {
    VT yv;
    row_cheb_next<VT, MT, PT>(A, sl.slot, sl.lane, wk, wprev, nullptr, y, theta, two_inv_eta, ck, 0, OffMat(), &yv);
    if (sl.lane == 0) {  // as k_multidot: v += z_j q_j from zero
      r = row_at(A, sl.slot);
      v[0] += (double)yv * (double)q[r];
    }
  }
  if (needs_stage(A)) tile_stage<1>(v, r >= 0 ? r - sl.tile * TPB : -1, stage);
  grid_sum_finish<1>(v, red, 1, sl.tile);
}

// The same with the outer iteration's window of products (y, q_i), i < k
// (q_i FP64), on any level (the finest: its row operands streamed, KIND): the
// sums of k_multidot<VT, double>.
template <typename VT, typename MT, typename PT, int KIND>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_next_mdot(Mat<MT> A, const VT* __restrict__ wk,
                                                                   const PT* wprev, VT* y, double theta,
                                                                   double two_inv_eta, double ck, VecPtrs qs, int k,
                                                                   Red red) {
  __shared__ double stage[8 * TPB];
  const SlotLane sl = slot_of(A);
  double v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.0;
  int r = -1;
  if (sl.slot >= 0) {
    VT yv;
    row_cheb_next<VT, MT, PT, KIND == kStepFine || KIND == kStepFineTimed>(A, sl.slot, sl.lane, wk, wprev, nullptr, y,
                                                                          theta, two_inv_eta, ck, 0, OffMat(), &yv);
    if (sl.lane == 0) {
      r = row_at(A, sl.slot);
      const double zj = (double)yv;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < k) v[i] += zj * static_cast<const double*>(qs.p[i])[r];
    }
  }
  if (needs_stage(A)) tile_stage<8>(v, r >= 0 ? r - sl.tile * TPB : -1, stage);
  grid_sum_finish<8>(v, red, k, sl.tile);
}

// degree 0: y = [y +] c0 w0
template <typename VT, typename RT>
__global__ void k_scale_add(int n, const RT* __restrict__ w0, VT* y, double c0, int accum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  VT v = (VT)c0 * (VT)w0[i];
  if (accum) v += y[i];
  y[i] = v;
}

template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_residual(Mat<MT> A, const RT* __restrict__ f,
                                                             const VT* __restrict__ x, VT* s) {
  const SlotLane q = slot_of(A);
  if (q.slot >= 0) (void)row_residual<VT, MT, RT>(A, q.slot, q.lane, f, x, s);
}

// s = f - A (x + P e)
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_residual_p(Mat<MT> A, const RT* __restrict__ f,
                                                               const VT* __restrict__ x, const VT* __restrict__ e,
                                                               const int* __restrict__ agg, VT* s) {
  const SlotLane q = slot_of(A);
  if (q.slot >= 0) (void)row_residual_p<VT, MT, RT>(A, q.slot, q.lane, f, x, e, agg, s);
}

// FP64 residual with its squared norm: s = f - A x, (s, s).
__global__ void __launch_bounds__(kMaxRowThreads) k_residual_dot(Mat<double> A, const double* __restrict__ f,
                                                                 const double* __restrict__ x, double* s, Red red) {
  __shared__ double stage[TPB];
  const SlotLane q = slot_of(A);
  double v[1] = {0.0};
  int r = -1;
  if (q.slot >= 0) {
    r = row_residual<double, double, double>(A, q.slot, q.lane, f, x, s);
    if (r >= 0) v[0] = s[r] * s[r];
  }
  if (needs_stage(A)) tile_stage<1>(v, r >= 0 ? r - q.tile * TPB : -1, stage);
  grid_sum_finish<1>(v, red);
}

template <typename VT>
__global__ void k_restrict(Transfer T, const VT* __restrict__ s, VT* b) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I < T.nc) row_restrict<VT>(T, I, s, b);
}

// The same sums for large aggregates (an independent set of A^k makes
// aggregates of tens to hundreds of rows): one wavefront per aggregate loads
// 64 members' values at once, so that members lying side by side share cache
// lines and the loads are not one thread's serial chain; every lane then adds
// the values in member order (broadcast by shuffles), as row_restrict does.
constexpr int kRestrictWaveMembers = 24;  // mean aggregate size from which it is used

template <typename VT>
__global__ void __launch_bounds__(256) k_restrict_wave(Transfer T, const VT* __restrict__ s, VT* b) {
  const int I = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  const int lane = (int)threadIdx.x & 63;
  if (I >= T.nc) return;  // uniform per wavefront
  const int k0 = T.member_off[I], k1 = T.member_off[I + 1];
  VT acc = 0;
  for (int c = k0; c < k1; c += 64) {
    const int k = c + lane;
    const VT v = k < k1 ? s[T.members[k]] : (VT)0;
    const int cnt = min(64, k1 - c);
    for (int t = 0; t < cnt; ++t) acc += __shfl(v, t, 64);
  }
  if (lane == 0) b[I] = acc;
}

// b = P^T (f - A x) in one pass on launch-bound levels: block k takes the
// aggregates agg_blk[k] .. agg_blk[k + 1] - 1 (at most TPB member rows, their
// member lists contiguous), K lanes compute each member row's residual (the
// value k_residual stores), the rows are staged in member order and each
// aggregate adds its members in order, as k_restrict does.  slot_of_row maps
// a row to its slot in sorted layouts (null otherwise).
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_restrict_residual(Mat<MT> A, Transfer T,
                                                                      const int* __restrict__ agg_blk,
                                                                      const int* __restrict__ slot_of_row,
                                                                      const RT* __restrict__ f,
                                                                      const VT* __restrict__ x, VT* b) {
  __shared__ VT stage[TPB];
  const int J0 = agg_blk[blockIdx.x], J1 = agg_blk[blockIdx.x + 1];
  const int m0 = T.member_off[J0], m1 = T.member_off[J1];
  const int m = threadIdx.x >> A.lk, lane = threadIdx.x & ((1 << A.lk) - 1);
  if (m0 + m < m1) {
    const int r = T.members[m0 + m];
    const int slot = slot_of_row ? slot_of_row[r] : r;
    const VT v = row_residual_value<VT, MT, RT>(A, slot, lane, f, x, r);
    if (lane == 0) stage[m] = v;
  }
  __syncthreads();
  for (int J = J0 + (int)threadIdx.x; J < J1; J += blockDim.x) {
    VT acc = 0;
    for (int k = T.member_off[J]; k < T.member_off[J + 1]; ++k) acc += stage[k - m0];
    b[J] = acc;
  }
}

// out = a x + b y in FP64 (out may alias x or y).
template <typename VT>
__global__ void k_axpby(int n, double a, const VT* x, double b, const VT* y, VT* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (VT)(a * (double)x[i] + b * (double)y[i]);
}

template <typename VT>
__global__ void k_prolong(Transfer T, const VT* __restrict__ e, VT* x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T.n) row_prolong<VT>(T, i, e, x);
}

template <typename VT, typename RT>
__global__ void __launch_bounds__(TPB) k_coarse_inv(CoarseView C, const RT* __restrict__ b, VT* x) {
  __shared__ double sb[1024], sy[1024];
  coarse_apply<VT, RT>(C, b, x, sb, sy);
}

// Substitution with the factor itself for coarsest levels above 1024 rows.
template <typename VT, typename RT>
__global__ void __launch_bounds__(TPB) k_coarse_subst(int n, const double* __restrict__ Lg, const RT* __restrict__ b,
                                                      VT* x) {
  extern __shared__ double y[];
  for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = (double)b[i];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double yk = y[k] / Lg[(size_t)k * n + k];
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) y[i] -= Lg[(size_t)i * n + k] * yk;
    if (threadIdx.x == 0) y[k] = yk;
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double xk = y[k] / Lg[(size_t)k * n + k];
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) y[i] -= Lg[(size_t)k * n + i] * xk;
    if (threadIdx.x == 0) y[k] = xk;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = (VT)y[i];
}

// (z, q_i) for i < k.
template <typename ZT, typename QT>
__global__ void __launch_bounds__(TPB) k_multidot(int n, const ZT* __restrict__ z, VecPtrs qs, int k, Red red) {
  double v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.0;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const double zj = (double)z[j];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < k) v[i] += zj * (double)static_cast<const QT*>(qs.p[i])[j];
  }
  grid_sum_finish<8>(v, red, k);
}

// p = z - sum_i (dots_i / rho_i) p_i  (term dropped when rho_i <= 0); FP64 arithmetic.
template <typename PT, typename ZT>
__global__ void __launch_bounds__(TPB) k_fcg_p(int n, PT* p, const ZT* z, VecPtrs ps, int k, const double* scal,
                                               Slots dots, Slots rhos) {
  double beta[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) beta[i] = i < k ? fcg_beta(scal, dots.s[i], rhos.s[i]) : 0.0;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double v = (double)z[j];
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < k) v = __builtin_fma(-beta[i], (double)static_cast<const PT*>(ps.p[i])[j], v);
  p[j] = (PT)v;
}

// q = A p; (p, q) and (p, r), added per tile in row order.
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_spmv_dots(Mat<MT> A, const VT* __restrict__ p, VT* q,
                                                              const RT* __restrict__ rv, Red red) {
  __shared__ double stage[2 * TPB];
  const SlotLane sl = slot_of(A);
  double v[2] = {0.0, 0.0};
  int r = -1;
  if (sl.slot >= 0) r = row_spmv_dots<VT, MT, RT>(A, sl.slot, sl.lane, p, q, rv, v);
  if (needs_stage(A)) tile_stage<2>(v, r >= 0 ? r - sl.tile * TPB : -1, stage);
  grid_sum_finish<2>(v, red);
}

// alpha = gamma / rho; x (= or +=) alpha p; optionally r -= alpha q and (r, r).
template <typename VT, typename PT, bool RR>
__global__ void __launch_bounds__(TPB) k_fcg_xr(int n, const PT* __restrict__ p, const VT* __restrict__ q, VT* x,
                                                VT* r, const double* scal, int s_rho, int s_gam, int x_init,
                                                int upd_r, Red red) {
  const double alpha = fcg_alpha(scal, s_rho, s_gam);
  double v[1] = {0.0};
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const double pj = (double)p[j];
    x[j] = x_init ? (VT)(alpha * pj) : fcg_axpy<VT>(alpha, pj, (double)x[j]);
    if (upd_r) {
      const double rj = __builtin_fma(-alpha, (double)q[j], (double)r[j]);
      r[j] = (VT)rj;
      if (RR) v[0] = rj * rj;
    }
  }
  if (RR) grid_sum_finish<1>(v, red);
}

// ---- flexible-CG updates folded into the kernels that read their results
// (inner solves of the launch-bound levels, two steps).

// First smoothing step of inner step 1 with step 0's update applied on the
// fly: w0 = rhs - alpha q (stored into rhs2 for the steps that follow) and
// sol = alpha p (x_init) or sol + alpha p.
template <typename VT, typename MT>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_first_upd(Mat<MT> A, const VT* __restrict__ rhs,
                                                                   const VT* __restrict__ q, VT* rhs2,
                                                                   const VT* __restrict__ p, VT* sol, int x_init,
                                                                   VT* w1, VT* y, double theta, double inv_eta,
                                                                   double c0, double c1, int store,
                                                                   double* scal, int s_rho, int s_gam,
                                                                   PendingSum pend) {
  double alpha;
  if (pend.nparts > 0) {  // rho and gamma still partials: finished here (slots s_rho, s_gam)
    double pv[2];
    finish_pending<2>(pend, scal, pv);
    alpha = fcg_alpha_of(pv[0], pv[1]);
  } else {
    alpha = fcg_alpha(scal, s_rho, s_gam);
  }
  const SlotLane sl = slot_of(A);
  if (sl.slot < 0) return;
  VT w0v;
  const int r = row_cheb_first_a<VT, MT>(A, sl.slot, sl.lane, XAxpy<VT>{rhs, q, alpha}, w1, y, YPlain<VT>{y}, theta,
                                         inv_eta, c0, c1, 0, store, &w0v);
  if (r >= 0) {
    rhs2[r] = w0v;
    const double pr = (double)p[r];
    sol[r] = x_init ? (VT)(alpha * pr) : fcg_axpy<VT>(alpha, pr, (double)sol[r]);
  }
}

// q = A p with p = z - beta z0 formed on the fly (beta = dot / rho) and
// stored into pout; (p, q) and (p, r) as in k_spmv_dots.
template <typename VT, typename MT>
__global__ void __launch_bounds__(kMaxRowThreads) k_spmv_dots_dir(Mat<MT> A, const VT* __restrict__ z,
                                                                  const VT* __restrict__ z0, VT* pout, VT* q,
                                                                  const VT* __restrict__ rv, double* scal,
                                                                  int s_dot, int s_rho, Red red, PendingSum pend) {
  __shared__ double stage[2 * TPB];
  double beta;
  if (pend.nparts > 0) {  // the dot still partials: finished here (slot s_dot)
    double pv[1];
    finish_pending<1>(pend, scal, pv);
    beta = fcg_beta_of(pv[0], scal[s_rho]);
  } else {
    beta = fcg_beta(scal, s_dot, s_rho);
  }
  const SlotLane sl = slot_of(A);
  double v[2] = {0.0, 0.0};
  int r = -1;
  if (sl.slot >= 0) {
    VT pr;
    r = row_spmv_dots_a<VT, MT, VT>(A, sl.slot, sl.lane, XDir<VT>{z, z0, beta}, q, rv, v, &pr);
    if (r >= 0) pout[r] = pr;
  }
  if (needs_stage(A)) tile_stage<2>(v, r >= 0 ? r - sl.tile * TPB : -1, stage);
  grid_sum_finish<2>(v, red);
}

// The prolongation consumers with the coarse correction e = esol + alpha ep
// (the inner solve's last update, never stored).
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_residual_pu(Mat<MT> A, const RT* __restrict__ f,
                                                                const VT* __restrict__ x, const VT* __restrict__ esol,
                                                                const VT* __restrict__ ep, const int* __restrict__ agg,
                                                                VT* s, const double* scal, int s_rho, int s_gam) {
  const double alpha = fcg_alpha(scal, s_rho, s_gam);
  const SlotLane q = slot_of(A);
  if (q.slot >= 0)
    (void)row_residual_a<VT, MT, RT>(A, q.slot, q.lane, f,
                                     XProlongC<VT, CUpd<VT>>{x, CUpd<VT>{esol, ep, alpha}, agg}, s);
}

template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(kMaxRowThreads) k_cheb_first_fu(Mat<MT> A, const RT* __restrict__ w0, VT* w1, VT* y,
                                                                  double theta, double inv_eta, double c0, double c1,
                                                                  int store, const VT* __restrict__ esol,
                                                                  const VT* __restrict__ ep, const int* __restrict__ agg,
                                                                  const double* scal, int s_rho, int s_gam) {
  const double alpha = fcg_alpha(scal, s_rho, s_gam);
  const SlotLane q = slot_of(A);
  if (q.slot < 0) return;
  VT w0v;
  (void)row_cheb_first_a<VT, MT>(A, q.slot, q.lane, XPlain<RT>{w0}, w1, y,
                                 YFold<VT, CUpd<VT>>{y, CUpd<VT>{esol, ep, alpha}, agg}, theta, inv_eta, c0, c1, 1,
                                 store, &w0v);
}

template <typename VT>
__global__ void k_prolong_u(Transfer T, const VT* __restrict__ esol, const VT* __restrict__ ep, VT* x,
                            const double* scal, int s_rho, int s_gam) {
  const double alpha = fcg_alpha(scal, s_rho, s_gam);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T.n) x[i] += CUpd<VT>{esol, ep, alpha}(T.agg[i]);
}

// Stores the two numbers of the host's stopping test (scal[a], scal[b]) into
// the pinned host mirror (system-scope stores, visible once the stream has
// been synchronized).
__device__ __forceinline__ void publish2(double* host, double va, double vb) {
  __hip_atomic_store(host + 1, vb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(host, va, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// host: also publish (acc[0], scal[pub]) for the host (K = 1 sums only).
template <int K>
__global__ void __launch_bounds__(kFinishThreads) k_finish_sum(int nparts, const double* partials, double* scal,
                                                               Slots slots, int kn, double* host, int pub) {
  __shared__ double red[16 * 8];
  double acc[K];
  sum_partials<K>(partials, nparts, acc, red, kn);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kn) scal[slots.s[k]] = acc[k];
    if (host) publish2(host, acc[0], scal[pub]);
  }
}

__global__ void k_publish(const double* scal, int a, int b, double* host) {
  if (threadIdx.x == 0) publish2(host, scal[a], scal[b]);
}

template <typename A, typename B>
__global__ void k_convert(int n, const A* __restrict__ a, B* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (B)a[i];
}

__global__ void k_zero_u32(unsigned* c) { *c = 0u; }

// ------------------------------------------------------------------ tail kernel
template <typename VT, typename MT>
__global__ void __launch_bounds__(TAIL_THREADS) k_tail(TailProgram P) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double red[16 * 8];
  __shared__ double sb[1024], sy[1024];
  run_tail<VT, MT>(P, lds, red, sb, sy, true);
}

// ------------------------------------------------------------------ host orchestration
Slots slots1(int a) {
  Slots s;
  for (int i = 0; i < 8; ++i) s.s[i] = S_DUMMY;
  s.s[0] = a;
  return s;
}
Slots slots2(int a, int b) {
  Slots s = slots1(a);
  s.s[1] = b;
  return s;
}
Slots slots_range(int base, int k) {
  Slots s;
  for (int i = 0; i < 8; ++i) s.s[i] = i < k ? base + i : S_DUMMY;
  return s;
}

// Builds the step sequence of the cycle.  With `rec` set, steps are appended
// to an op program for the tail interpreter instead of being launched.
template <typename VT, typename MT>
struct Engine {
  amg_hier* h;
  hipStream_t s;
  std::vector<TailOp>* rec = nullptr;
  // Reduction scratch: the scalar area, the block partials and the arrival
  // counter -- the hierarchy's own buffers unless a solve supplies others.
  double* scal_ = nullptr;
  double* partials_ = nullptr;
  unsigned* counter_ = nullptr;
  double* sc() const { return scal_ ? scal_ : h->scal; }
  double* pa() const { return partials_ ? partials_ : h->partials; }
  unsigned* co() const { return counter_ ? counter_ : h->counter; }

  // An inner solve's last update x += alpha p, left to the kernels that read
  // the coarse correction (alpha from the step's scalar slots).
  struct Deferred {
    bool on = false;
    const VT* sol = nullptr;
    const VT* p = nullptr;
    int s_rho = 0, s_gam = 0;
  };
  // The previous inner step's update, applied by the first smoothing step of
  // the next one: rhs2 = rhs - alpha q, sol = [sol +] alpha p.
  struct StepUpd {
    const VT* rhs;
    const VT* q;
    const VT* p;
    VT* sol;
    int x_init;
    int s_rho, s_gam;
    PendingSum pend;  // rho and gamma left as partials (nparts 0: in scal)
  };
  // The inner product (result, q) into scal[slot], asked of a cycle so that
  // its last smoothing step can form it (done is set when it did; pend holds
  // its partials when their finish is left to the next kernel).
  struct DotReq {
    const VT* q;
    int slot;
    bool done;
    PendingSum pend;
  };
  // The outer iteration's window of products (result, q_i), i < k (q_i FP64),
  // into slots, asked of the finest level's cycle in the same way.
  struct MDotReq {
    VecPtrs qs;
    int k;
    Slots slots;
    bool done;
  };

  Mat<MT> A(int l) const { return mat_of<MT>(h->lv[l]); }
  static VT* wsv(void* p) { return static_cast<VT*>(p); }

  static TailOp op(int type, int level, int n) {
    TailOp o;
    std::memset(&o, 0, sizeof(o));
    o.type = type;
    o.level = level;
    o.n = n;
    return o;
  }

  // reduction destination for a device-wide kernel of `blocks` blocks
  Red red_for(int blocks, Slots slots) const {
    return Red{pa(), co(), sc(), slots, blocks <= h->last_block_max ? 1 : 0};
  }
  // A reduction of `blocks` blocks (K values each) whose finish the next
  // kernel takes over: too many blocks to finish in the kernel, and its
  // partials fit the upper half of the partials buffer (the lower half stays
  // for the consumer's own reduction).
  bool defer_finish(int blocks, int K) const {
    return !rec && blocks > h->last_block_max && (size_t)blocks * K <= (size_t)h->max_blocks * 4;
  }
  double* pa_deferred() const { return pa() + (size_t)h->max_blocks * 4; }
  // host: publish (the sum, scal[pub]) to the pinned host mirror as well
  template <int K>
  int32_t finish(int blocks, Slots slots, double* host = nullptr, int pub = 0, int kn = K) {
    if (blocks <= h->last_block_max) {
      if (host) {
        hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, (const double*)sc(), slots.s[0], pub, host);
        AMG_HIP(hipGetLastError());
      }
      return AMG_OK;
    }
    hipLaunchKernelGGL((k_finish_sum<K>), dim3(1), dim3(kFinishThreads), 0, s, blocks, pa(), sc(), slots,
                       kn, host, pub);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // fold_e: y holds x before the prolongation of the coarse correction fold_e
  // (fold_d.on: the correction is fold_d.sol + alpha fold_d.p).  upd: w0 is
  // rhs2 of the update, formed on the fly and stored (accum false).
  template <typename RT>
  int32_t cheb_first(int l, const RT* w0, VT* w1, VT* y, double c0, double c1, bool accum, bool store,
                     const VT* fold_e = nullptr, const Deferred* fold_d = nullptr, const StepUpd* upd = nullptr) {
    const Level& lv = h->lv[l];
    if (!rec && upd) {
      if constexpr (std::is_same<RT, VT>::value) {
        const auto Am = A(l);
        hipLaunchKernelGGL((k_cheb_first_upd<VT, MT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, upd->rhs, upd->q,
                           const_cast<VT*>(w0), upd->p, upd->sol, upd->x_init, w1, y, lv.theta, 1.0 / lv.eta, c0, c1,
                           (int)store, sc(), upd->s_rho, upd->s_gam, upd->pend);
        AMG_HIP(hipGetLastError());
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    if (!rec && fold_d && fold_d->on) {
      const auto Am = A(l);
      hipLaunchKernelGGL((k_cheb_first_fu<VT, MT, RT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, w0, w1, y, lv.theta,
                         1.0 / lv.eta, c0, c1, (int)store, fold_d->sol, fold_d->p, transfer_of(h, l).agg,
                         (const double*)sc(), fold_d->s_rho, fold_d->s_gam);
      AMG_HIP(hipGetLastError());
      return AMG_OK;
    }
    if (rec) {
      if constexpr (std::is_same<RT, VT>::value) {
        TailOp o = op(OP_CHEB_FIRST, l, lv.n);
        o.a = w0; o.c = w1; o.d = y;
        o.f0 = lv.theta; o.f1 = 1.0 / lv.eta; o.f2 = c0; o.f3 = c1;
        o.i0 = accum; o.i1 = store;
        if (fold_e) {
          o.i2 = 1;
          o.k = 1;
          o.w.p[0] = fold_e;
        }
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    const auto Am = A(l);
    const int* agg = fold_e ? transfer_of(h, l).agg : nullptr;
    hipLaunchKernelGGL((k_cheb_first<VT, MT, RT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, w0, w1, y, lv.theta,
                       1.0 / lv.eta, c0, c1, (int)accum, (int)store, fold_e, agg);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  template <typename PT>
  int32_t cheb_next(int l, const VT* wk, const PT* wprev, VT* wnext, VT* y, double ck, bool store) {
    const Level& lv = h->lv[l];
    if (rec) {
      if constexpr (std::is_same<PT, VT>::value) {
        TailOp o = op(OP_CHEB_NEXT, l, lv.n);
        o.a = wk; o.b = wprev; o.c = wnext; o.d = y;
        o.f0 = lv.theta; o.f1 = 2.0 / lv.eta; o.f2 = ck;
        o.i0 = store;
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    const auto Am = A(l);
    const double ti = 2.0 / lv.eta;
    if (l == 0 && lv.n >= kStreamRows) {
      if (store)
        hipLaunchKernelGGL((k_cheb_next<VT, MT, PT, true, kStepFine>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wprev, wnext,
                           y, lv.theta, ti, ck);
      else
        hipLaunchKernelGGL((k_cheb_next<VT, MT, PT, false, kStepFine>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wprev,
                           wnext, y, lv.theta, ti, ck);
    } else {
      if (store)
        hipLaunchKernelGGL((k_cheb_next<VT, MT, PT, true, kStepCoarse>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wprev,
                           wnext, y, lv.theta, ti, ck);
      else
        hipLaunchKernelGGL((k_cheb_next<VT, MT, PT, false, kStepCoarse>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wprev,
                           wnext, y, lv.theta, ti, ck);
    }
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // the last step of a smoothing (nothing stored but y) with (y, dot->q)
  template <typename PT>
  int32_t cheb_next_dot(int l, const VT* wk, const PT* wprev, VT* y, double ck, DotReq* dot) {
    const Level& lv = h->lv[l];
    const auto Am = A(l);
    const Slots sl = slots1(dot->slot);
    const bool defer = defer_finish(Am.nb, 1);
    const Red rd = defer ? Red{pa_deferred(), co(), sc(), sl, 0} : red_for(Am.nb, sl);
    hipLaunchKernelGGL((k_cheb_next_dot<VT, MT, PT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wprev, y,
                       lv.theta, 2.0 / lv.eta, ck, dot->q, rd);
    AMG_HIP(hipGetLastError());
    if (defer) {
      dot->pend = PendingSum{pa_deferred(), Am.nb, 1, sl};
    } else {
      AMG_TRY(finish<1>(Am.nb, sl));
    }
    dot->done = true;
    return AMG_OK;
  }

  // the last step of a smoothing with the window products (y, q_i)
  template <typename PT>
  int32_t cheb_next_mdot(int l, const VT* wk, const PT* wprev, VT* y, double ck, MDotReq* md) {
    const Level& lv = h->lv[l];
    const auto Am = A(l);
    const double ti = 2.0 / lv.eta;
    const Red rd = red_for(Am.nb, md->slots);
    if (l == 0 && lv.n >= kStreamRows)
      hipLaunchKernelGGL((k_cheb_next_mdot<VT, MT, PT, kStepFine>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk,
                         wprev, y, lv.theta, ti, ck, md->qs, md->k, rd);
    else
      hipLaunchKernelGGL((k_cheb_next_mdot<VT, MT, PT, kStepCoarse>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk,
                         wprev, y, lv.theta, ti, ck, md->qs, md->k, rd);
    AMG_HIP(hipGetLastError());
    AMG_TRY(finish<8>(Am.nb, md->slots, nullptr, 0, md->k));
    md->done = true;
    return AMG_OK;
  }

  // `reps` back-to-back launches of the finest level's storing Chebyshev step
  // (w_k fixed in buffer A, w_{k-1} and w_{k+1} in buffer B, y in S) between
  // two events; values stay bounded (B alternates between two vectors).
  int32_t time_fine_step(int reps, hipEvent_t e0, hipEvent_t e1) {
    const Level& lv = h->lv[0];
    const auto Am = A(0);
    VT* wk = wsv(h->ws[0].A);
    VT* wb = wsv(h->ws[0].B);
    VT* y = wsv(h->ws[0].S);
    const bool big = lv.n >= kStreamRows;  // the instance the solve launches
    AMG_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) {
      if (big)
        hipLaunchKernelGGL((k_cheb_next<VT, MT, VT, true, kStepFine>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk, wb,
                           wb, y, lv.theta, 2.0 / lv.eta, 1e-3);
      else
        hipLaunchKernelGGL((k_cheb_next<VT, MT, VT, true, kStepCoarse>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, wk,
                           wb, wb, y, lv.theta, 2.0 / lv.eta, 1e-3);
    }
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipEventRecord(e1, s));
    return AMG_OK;
  }

  // `reps` back-to-back launches of the same step cycling over nc copies of
  // the finest level (matrix, diagonal and the three vectors; copy i % nc for
  // launch i), so that each launch streams its data from HBM: with the copies
  // together well above the 256 MB Infinity Cache, a copy has been displaced
  // by the others before it comes round again.  One untimed round first.
  int32_t time_fine_step_rotating(int reps, int nc, const Mat<MT>* mats, VT* const* wk, VT* const* wb, VT* const* y,
                                  hipEvent_t e0, hipEvent_t e1) {
    const Level& lv = h->lv[0];
    const bool big = lv.n >= kStreamRows;
    for (int i = 0; i < reps + nc; ++i) {
      if (i == nc) AMG_HIP(hipEventRecord(e0, s));
      const int c = i % nc;
      if (big)
        hipLaunchKernelGGL((k_cheb_next<VT, MT, VT, true, kStepFineTimed>), dim3(mats[c].nb), dim3(TPB << mats[c].lk),
                           0, s, mats[c], wk[c], wb[c], wb[c], y[c], lv.theta, 2.0 / lv.eta, 1e-3);
      else
        hipLaunchKernelGGL((k_cheb_next<VT, MT, VT, true, kStepSmallTimed>), dim3(mats[c].nb), dim3(TPB << mats[c].lk),
                           0, s, mats[c], wk[c], wb[c], wb[c], y[c], lv.theta, 2.0 / lv.eta, 1e-3);
    }
    AMG_HIP(hipGetLastError());
    AMG_HIP(hipEventRecord(e1, s));
    return AMG_OK;
  }

  template <typename RT>
  int32_t scale_add(int l, const RT* w0, VT* y, double c0, bool accum) {
    const int n = h->lv[l].n;
    if (rec) {
      if constexpr (std::is_same<RT, VT>::value) {
        TailOp o = op(OP_SCALE_ADD, l, n);
        o.a = w0; o.d = y; o.f0 = c0; o.i0 = accum;
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    hipLaunchKernelGGL((k_scale_add<VT, RT>), dim3(nblk(n)), dim3(TPB), 0, s, n, w0, y, c0, (int)accum);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // y = [y +] q_m(A_l) r: m three-term steps; buffers A, B of the level hold
  // w_k and w_{k-1} (w_{k+1} overwrites w_{k-1} in place).  fold_e (m >= 1,
  // accumulating): y is x before the prolongation x += P fold_e.
  template <typename RT>
  int32_t smooth(int l, const RT* r, VT* y, bool accum, const VT* fold_e = nullptr, const Deferred* fold_d = nullptr,
                 const StepUpd* upd = nullptr, DotReq* dot = nullptr, MDotReq* mdot = nullptr) {
    const Level& lv = h->lv[l];
    const int m = h->p.degree;
    const double* c = lv.coef.data();
    if (m == 0) return scale_add(l, r, y, c[0], accum);
    VT* bufA = wsv(h->ws[l].A);
    VT* bufB = wsv(h->ws[l].B);
    AMG_TRY(cheb_first(l, r, bufA, y, c[0], c[1], accum, m > 1, fold_e, fold_d, upd));
    VT* cur = bufA;
    VT* prevbuf = nullptr;
    for (int k = 1; k < m; ++k) {
      const bool store = (k + 1 < m);
      const bool with_dot = dot && !rec && !store;
      const bool with_mdot = mdot && !rec && !store;
      VT* next;
      if (k == 1) {
        next = bufB;
        if (with_dot)
          AMG_TRY(cheb_next_dot(l, cur, r, y, c[k + 1], dot));
        else if (with_mdot)
          AMG_TRY(cheb_next_mdot(l, cur, r, y, c[k + 1], mdot));
        else
          AMG_TRY(cheb_next(l, cur, r, next, y, c[k + 1], store));
      } else {
        next = prevbuf;
        if (with_dot)
          AMG_TRY(cheb_next_dot(l, cur, static_cast<const VT*>(prevbuf), y, c[k + 1], dot));
        else if (with_mdot)
          AMG_TRY(cheb_next_mdot(l, cur, static_cast<const VT*>(prevbuf), y, c[k + 1], mdot));
        else
          AMG_TRY(cheb_next(l, cur, static_cast<const VT*>(prevbuf), next, y, c[k + 1], store));
      }
      prevbuf = cur;
      cur = next;
    }
    return AMG_OK;
  }

  template <typename RT>
  int32_t residual(int l, const RT* f, const VT* x, VT* out) {
    if (rec) {
      if constexpr (std::is_same<RT, VT>::value) {
        TailOp o = op(OP_RESIDUAL, l, h->lv[l].n);
        o.a = f; o.b = x; o.c = out;
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    const auto Am = A(l);
    hipLaunchKernelGGL((k_residual<VT, MT, RT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, f, x, out);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // out = f - A (x + P e), x itself unchanged
  template <typename RT>
  int32_t residual_p(int l, const RT* f, const VT* x, const VT* e, VT* out, const Deferred* d = nullptr) {
    if (!rec && d && d->on) {
      const auto Am = A(l);
      hipLaunchKernelGGL((k_residual_pu<VT, MT, RT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, f, x, d->sol, d->p,
                         transfer_of(h, l).agg, out, (const double*)sc(), d->s_rho, d->s_gam);
      AMG_HIP(hipGetLastError());
      return AMG_OK;
    }
    if (rec) {
      if constexpr (std::is_same<RT, VT>::value) {
        TailOp o = op(OP_RESIDUAL_P, l, h->lv[l].n);
        o.a = f; o.b = x; o.c = out;
        o.k = 1;
        o.w.p[0] = e;
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    const auto Am = A(l);
    hipLaunchKernelGGL((k_residual_p<VT, MT, RT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, f, x, e,
                       transfer_of(h, l).agg, out);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // b = P^T (f - A x) without storing the residual (levels with an
  // aggregate-to-block map); false when the level has none.
  template <typename RT>
  bool restrict_residual(int l, const RT* f, const VT* x, VT* b, int32_t* st) {
    const auto& W = h->ws[l];
    if (rec || !h->p.fuse || !W.agg_blk) return false;
    const auto Am = A(l);
    hipLaunchKernelGGL((k_restrict_residual<VT, MT, RT>), dim3(W.n_agg_blk), dim3(TPB << Am.lk), 0, s, Am,
                       transfer_of(h, l), (const int*)W.agg_blk, (const int*)W.slot_of_row, f, x, b);
    const hipError_t e = hipGetLastError();
    *st = e == hipSuccess ? AMG_OK : AMG_ERR_DEVICE;
    if (e != hipSuccess) set_last_error(std::string("k_restrict_residual: ") + hipGetErrorString(e));
    return true;
  }

  int32_t restrict_(int l, const VT* sv, VT* b) {
    const Transfer T = transfer_of(h, l);
    if (rec) {
      TailOp o = op(OP_RESTRICT, l, T.nc);
      o.a = sv; o.c = b;
      rec->push_back(o);
      return AMG_OK;
    }
    if (T.n >= kRestrictWaveMembers * (int64_t)T.nc)
      hipLaunchKernelGGL((k_restrict_wave<VT>), dim3((T.nc + 3) / 4), dim3(256), 0, s, T, sv, b);
    else
      hipLaunchKernelGGL((k_restrict<VT>), dim3(nblk(T.nc)), dim3(TPB), 0, s, T, sv, b);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  int32_t prolong(int l, const VT* e, VT* x, const Deferred* d = nullptr) {
    const Transfer T = transfer_of(h, l);
    if (!rec && d && d->on) {
      hipLaunchKernelGGL((k_prolong_u<VT>), dim3(nblk(T.n)), dim3(TPB), 0, s, T, d->sol, d->p, x,
                         (const double*)sc(), d->s_rho, d->s_gam);
      AMG_HIP(hipGetLastError());
      return AMG_OK;
    }
    if (rec) {
      TailOp o = op(OP_PROLONG, l, T.n);
      o.a = e; o.c = x;
      rec->push_back(o);
      return AMG_OK;
    }
    hipLaunchKernelGGL((k_prolong<VT>), dim3(nblk(T.n)), dim3(TPB), 0, s, T, e, x);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  template <typename RT>
  int32_t coarse(const RT* b, VT* x) {
    const int n = h->nL;
    if (rec) {
      if constexpr (std::is_same<RT, VT>::value) {
        TailOp o = op(OP_COARSE, h->L, n);
        o.a = b; o.c = x;
        rec->push_back(o);
        return AMG_OK;
      }
      return AMG_ERR_DEVICE;
    }
    if (h->chol_inv) {
      const CoarseView C{n, h->chol_inv, h->chol_invT};
      hipLaunchKernelGGL((k_coarse_inv<VT, RT>), dim3(1), dim3(TPB), 0, s, C, b, x);
    } else {
      hipLaunchKernelGGL((k_coarse_subst<VT, RT>), dim3(1), dim3(TPB), sizeof(double) * n, s, n, h->chol, b, x);
    }
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // (z, q_i), i < k; z of the cycle vector type, q_i of the cycle type
  // (coarse levels) or FP64 (outer window)
  int32_t multidot(int level, int n, const void* z, const VecPtrs& qs, int k, Slots out, bool q_fp64) {
    if (rec) {
      TailOp o = op(OP_MULTIDOT, level, n);
      o.a = z; o.w = qs; o.k = k; o.s0 = out;
      rec->push_back(o);
      return AMG_OK;
    }
    const int nb = nblk(n);
    const Red rd = red_for(nb, out);
    if (q_fp64) {
      hipLaunchKernelGGL((k_multidot<VT, double>), dim3(nb), dim3(TPB), 0, s, n, (const VT*)z, qs, k, rd);
    } else {
      hipLaunchKernelGGL((k_multidot<VT, VT>), dim3(nb), dim3(TPB), 0, s, n, (const VT*)z, qs, k, rd);
    }
    AMG_HIP(hipGetLastError());
    return finish<8>(nb, out, nullptr, 0, k);
  }

  // -------- flexible CG steps on a coarse level (cycle vector type)
  int32_t spmv_dots(int l, const VT* p, VT* q, const VT* rv, Slots out) {
    if (rec) {
      TailOp o = op(OP_SPMV_DOTS, l, h->lv[l].n);
      o.a = p; o.b = rv; o.c = q; o.s0 = out;
      rec->push_back(o);
      return AMG_OK;
    }
    const auto Am = A(l);
    hipLaunchKernelGGL((k_spmv_dots<VT, MT, VT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, p, q, rv, red_for(Am.nb, out));
    AMG_HIP(hipGetLastError());
    return finish<2>(Am.nb, out);
  }

  int32_t fcg_p(int l, int n, VT* p, const VT* z, const VecPtrs& ps, int k, Slots dots, Slots rhos) {
    if (rec) {
      TailOp o = op(OP_FCG_P, l, n);
      o.a = z; o.c = p; o.w = ps; o.k = k; o.s0 = dots; o.s1 = rhos;
      rec->push_back(o);
      return AMG_OK;
    }
    hipLaunchKernelGGL((k_fcg_p<VT, VT>), dim3(nblk(n)), dim3(TPB), 0, s, n, p, z, ps, k, sc(), dots, rhos);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  int32_t fcg_xr(int l, int n, const VT* p, const VT* q, VT* x, VT* r, int s_rho, int s_gam, bool x_init,
                 bool upd_r) {
    if (rec) {
      TailOp o = op(OP_FCG_XR, l, n);
      o.a = p; o.b = q; o.c = x; o.d = r;
      o.i0 = s_rho; o.i1 = s_gam; o.i2 = x_init; o.i3 = upd_r;
      rec->push_back(o);
      return AMG_OK;
    }
    const int nb = nblk(n);
    hipLaunchKernelGGL((k_fcg_xr<VT, VT, false>), dim3(nb), dim3(TPB), 0, s, n, p, q, x, r, sc(), s_rho, s_gam,
                       (int)x_init, (int)upd_r, red_for(nb, slots1(S_DUMMY)));
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // the recorded inner solve of the tail level, in one workgroup
  int32_t tail() {
    hipLaunchKernelGGL((k_tail<VT, MT>), dim3(1), dim3(h->tail_threads), h->tail_lds_bytes, s,
                       *static_cast<const TailProgram*>(h->tail_prog));
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // x = Kcycle(l, r)
  template <typename RT>
  // upd: the first smoothing step also applies the previous inner step's
  // update (r is then the rhs2 it writes).
  int32_t kcycle(int l, const RT* r, VT* x, const StepUpd* upd = nullptr, DotReq* dot = nullptr,
                 MDotReq* mdot = nullptr) {
    if (l == h->L) return coarse(r, x);
    VT* S = wsv(h->ws[l].S);
    VT* b = wsv(h->ws[l + 1].rhs);
    VT* e = wsv(h->ws[l + 1].sol);
    AMG_TRY(smooth(l, r, x, false, nullptr, nullptr, upd));
    int32_t rst = AMG_OK;
    if (restrict_residual(l, r, x, b, &rst)) {
      AMG_TRY(rst);
    } else {
      AMG_TRY(residual(l, r, x, S));
      AMG_TRY(restrict_(l, S, b));
    }
    Deferred d;
    if (l + 1 == h->L) {
      AMG_TRY(coarse(static_cast<const VT*>(b), e));
    } else if (!rec && h->tail_level == l + 1) {
      AMG_TRY(tail());
    } else if (h->p.cycle == AMG_CYCLE_AMLI) {
      AMG_TRY(amli_correction(l + 1));
    } else {
      AMG_TRY(inner(l + 1, &d));
    }
    // on launch-bound levels (and in recorded programs) the prolongation
    // x += P e is folded into the residual and the first smoothing step that
    // follow it: the same roundings, one pass fewer
    if (h->p.degree > 0 && (rec || h->lv[l].n < kFoldProlongRows)) {
      AMG_TRY(residual_p(l, r, x, e, S, &d));
      AMG_TRY(smooth(l, static_cast<const VT*>(S), x, true, e, &d, nullptr, dot, mdot));
      return AMG_OK;
    }
    AMG_TRY(prolong(l, e, x, &d));
    AMG_TRY(residual(l, r, x, S));
    AMG_TRY(smooth(l, static_cast<const VT*>(S), x, true, nullptr, nullptr, nullptr, dot, mdot));
    return AMG_OK;
  }

  // The coarse correction of the cycle on level l (1 <= l < L): rhs -> sol.
  int32_t coarse_correction(int l) {
    if (h->p.cycle == AMG_CYCLE_AMLI) return amli_correction(l);
    return inner(l);
  }

  // Stationary AMLI: sol = g0 y0 + g1 B(A y0), y0 = B rhs, with B the cycle on
  // level l and g0 + g1 t the degree-1 best approximation to 1/t on [a_l, 1].
  int32_t amli_correction(int l) {
    auto& W = h->ws[l];
    VT* rhs = wsv(W.rhs);
    VT* sol = wsv(W.sol);
    VT* y0 = wsv(W.Z[0]);
    VT* y1 = wsv(W.Z[1]);
    VT* ay = wsv(W.Q[0]);
    if ((int)h->amli_g0.size() <= l) {
      set_last_error("AMLI coefficients missing for level " + std::to_string(l));
      return AMG_ERR_DEVICE;
    }
    AMG_TRY(kcycle(l, static_cast<const VT*>(rhs), y0));
    AMG_TRY(spmv_dots(l, y0, ay, y0, slots2(S_DUMMY, S_DUMMY)));
    AMG_TRY(kcycle(l, static_cast<const VT*>(ay), y1));
    AMG_TRY(scale_add(l, static_cast<const VT*>(y0), sol, h->amli_g0[l], false));
    AMG_TRY(scale_add(l, static_cast<const VT*>(y1), sol, h->amli_g1[l], true));
    return AMG_OK;
  }

  // Two flexible-CG steps on a launch-bound level with the vector updates
  // folded into the kernels that read them: step 0's update goes into step
  // 1's first smoothing step, step 1's direction into its product, and step
  // 1's update of the solution into the caller's prolongation (*out).
  int32_t inner_folded(int l, Deferred* out) {
    const int n = h->lv[l].n;
    auto& W = h->ws[l];
    VT* rhs = wsv(W.rhs);
    VT* rhs2 = wsv(W.rhs2);
    VT* sol = wsv(W.sol);
    VT* Z0 = wsv(W.Z[0]);
    VT* Z1 = wsv(W.Z[1]);
    VT* Q0 = wsv(W.Q[0]);
    VT* Q1 = wsv(W.Q[1]);
    VT* P1 = wsv(W.P1);
    const int base = lbase(l);
    AMG_TRY(kcycle(l, static_cast<const VT*>(rhs), Z0));
    const auto Am = A(l);
    // step 0's (p, q) and (p, r): on a grid too large to finish them in the
    // kernel, the next cycle's first kernel (the only reader) finishes them
    StepUpd u{rhs, Q0, Z0, sol, 1, base, base + 8};
    const Slots pr0 = slots2(base, base + 8);
    if (defer_finish(Am.nb, 2)) {
      hipLaunchKernelGGL((k_spmv_dots<VT, MT, VT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, Z0, Q0, rhs,
                         Red{pa_deferred(), co(), sc(), pr0, 0});
      AMG_HIP(hipGetLastError());
      u.pend = PendingSum{pa_deferred(), Am.nb, 2, pr0};
    } else {
      AMG_TRY(spmv_dots(l, Z0, Q0, rhs, pr0));
    }
    // (Z1, Q0) from the cycle's last smoothing step when it can form it
    DotReq dq{Q0, base + 16, false, PendingSum{}};
    AMG_TRY(kcycle(l, static_cast<const VT*>(rhs2), Z1, &u, &dq));
    if (!dq.done) {
      VecPtrs qs{};
      qs.p[0] = W.Q[0];
      AMG_TRY(multidot(l, n, Z1, qs, 1, slots_range(base + 16, 1), false));
    }
    const Slots pq = slots2(base + 1, base + 9);
    hipLaunchKernelGGL((k_spmv_dots_dir<VT, MT>), dim3(Am.nb), dim3(TPB << Am.lk), 0, s, Am, Z1, Z0, P1, Q1, rhs2,
                       sc(), base + 16, base, red_for(Am.nb, pq), dq.pend);
    AMG_HIP(hipGetLastError());
    AMG_TRY(finish<2>(Am.nb, pq));
    out->on = true;
    out->sol = sol;
    out->p = P1;
    out->s_rho = base + 1;
    out->s_gam = base + 9;
    return AMG_OK;
  }

  // exactly nu flexible-CG steps from zero on level l (1 <= l < L): rhs -> sol
  // (with `out` given, the launch-bound two-step case may leave the last
  // update of sol to the caller, see inner_folded)
  int32_t inner(int l, Deferred* out = nullptr) {
    const int nu = h->p.inner_steps;
    if (out && !rec && h->p.fuse && nu == 2 && h->p.degree > 0 && h->lv[l].n < kFoldProlongRows && h->ws[l].rhs2 &&
        h->ws[l].P1)
      return inner_folded(l, out);
    const int n = h->lv[l].n;
    auto& W = h->ws[l];
    VT* rhs = wsv(W.rhs);
    VT* sol = wsv(W.sol);
    const int base = lbase(l);
    for (int k = 0; k < nu; ++k) {
      VT* z = wsv(W.Z[k]);
      AMG_TRY(kcycle(l, static_cast<const VT*>(rhs), z));
      if (k > 0) {
        VecPtrs qs{}, ps{};
        for (int i = 0; i < k; ++i) {
          qs.p[i] = W.Q[i];
          ps.p[i] = W.Z[i];
        }
        AMG_TRY(multidot(l, n, z, qs, k, slots_range(base + 16, k), false));
        AMG_TRY(fcg_p(l, n, z, z, ps, k, slots_range(base + 16, k), slots_range(base, k)));
      }
      VT* q = wsv(W.Q[k]);
      AMG_TRY(spmv_dots(l, z, q, rhs, slots2(base + k, base + 8 + k)));
      AMG_TRY(fcg_xr(l, n, z, q, sol, rhs, base + k, base + 8 + k, k == 0, k + 1 < nu));
    }
    return AMG_OK;
  }

  // Pinned host slots of the stopping test's two numbers, one pair per
  // window position, so that two iterations in flight never share one.
  double* pub_slot(int j) const { return h->host_scal + kPubBase + 2 * j; }

  // one outer iteration at window position j; u, r FP64 (finest level)
  int32_t outer_iter(int j, double* u) {
    const int n = h->lv[0].n;
    const int nb = nblk(n);
    const auto A64 = mat_of<double>(h->lv[0]);
    VT* z = wsv(h->z);
    VecPtrs qs{}, ps{};
    for (int i = 0; i < j; ++i) {
      qs.p[i] = h->Qo[i];
      ps.p[i] = h->P[i];
    }
    // the window products (z, q_i) from the cycle's last smoothing step when
    // it can form them
    MDotReq md{qs, j, slots_range(S_DOTS, j), false};
    AMG_TRY(kcycle(0, static_cast<const double*>(h->r), z, nullptr, nullptr, h->p.fuse && j > 0 ? &md : nullptr));
    if (j > 0 && !md.done) AMG_TRY(multidot(0, n, z, qs, j, slots_range(S_DOTS, j), true));
    hipLaunchKernelGGL((k_fcg_p<double, VT>), dim3(nb), dim3(TPB), 0, s, n, h->P[j], z, ps, j, sc(),
                       slots_range(S_DOTS, j), slots_range(S_RHOW, j));
    const Slots pq = slots2(S_RHOW + j, S_GAM);
    hipLaunchKernelGGL((k_spmv_dots<double, double, double>), dim3(A64.nb), dim3(TPB << A64.lk), 0, s, A64, h->P[j], h->Qo[j],
                       h->r, red_for(A64.nb, pq));
    AMG_TRY(finish<2>(A64.nb, pq));
    const Slots rr = slots1(S_RR);
    hipLaunchKernelGGL((k_fcg_xr<double, double, true>), dim3(nb), dim3(TPB), 0, s, n, h->P[j], h->Qo[j], u, h->r,
                       sc(), S_RHOW + j, S_GAM, 0, 1, red_for(nb, rr));
    AMG_HIP(hipGetLastError());
    if (h->p.stop == AMG_STOP_ENERGY) {
      // f = 0: the error is u itself; (u, A u) from a fresh product (the
      // recursive residual drifts along the constants of a Neumann problem,
      // which the iterates pick up), published with rho_j
      AMG_TRY(finish<1>(nb, rr));
      return energy64(u, pub_slot(j), S_RHOW + j);
    }
    // with the stopping test's inputs, (r, r) and rho_j, published to the host
    AMG_TRY(finish<1>(nb, rr, pub_slot(j), S_RHOW + j));
    return AMG_OK;
  }

  // (u, A u) into scal[S_XR] (A u into tmp); host: publish it with scal[pub]
  int32_t energy64(const double* u, double* host = nullptr, int pub = 0) {
    const auto A64 = mat_of<double>(h->lv[0]);
    const Slots sl = slots2(S_XR, S_DUMMY);
    hipLaunchKernelGGL((k_spmv_dots<double, double, double>), dim3(A64.nb), dim3(TPB << A64.lk), 0, s, A64, u,
                       h->tmp, u, red_for(A64.nb, sl));
    AMG_HIP(hipGetLastError());
    return finish<2>(A64.nb, sl, host, pub);
  }

  // (a, b) in FP64 into scal[slot] (finest-level vectors)
  int32_t dot64(const double* a, const double* b, int slot) {
    const int n = h->lv[0].n, nb = nblk(n);
    VecPtrs qs{};
    qs.p[0] = b;
    const Slots sl = slots1(slot);
    hipLaunchKernelGGL((k_multidot<double, double>), dim3(nb), dim3(TPB), 0, s, n, a, qs, 1, red_for(nb, sl));
    AMG_HIP(hipGetLastError());
    return finish<1>(nb, sl);
  }

  // out = f - A u (FP64) and its squared norm into scal[slot]
  int32_t residual64(const double* f, const double* u, double* out, int slot) {
    const auto A64 = mat_of<double>(h->lv[0]);
    const Slots sl = slots1(slot);
    hipLaunchKernelGGL(k_residual_dot, dim3(A64.nb), dim3(TPB << A64.lk), 0, s, A64, f, u, out, red_for(A64.nb, sl));
    AMG_HIP(hipGetLastError());
    return finish<1>(A64.nb, sl);
  }
};

using clk = std::chrono::steady_clock;

template <typename VT, typename MT>
int32_t capture_graphs(amg_hier* h, double* u) {
  // graphs are recorded with the solution pointer u baked in; re-record when it changes
  destroy_graphs(h);
  if (!h->graph_stream) AMG_HIP(hipStreamCreateWithFlags(&h->graph_stream, hipStreamNonBlocking));
  Engine<VT, MT> E{h, h->graph_stream};
  for (int j = 0; j < h->p.restart; ++j) {
    hipGraph_t g = nullptr;
    AMG_HIP(hipStreamBeginCapture(h->graph_stream, hipStreamCaptureModeThreadLocal));
    int32_t st = E.outer_iter(j, u);
    hipError_t e = hipStreamEndCapture(h->graph_stream, &g);
    if (st != AMG_OK) return st;
    AMG_HIP(e);
    e = hipGraphInstantiate(&h->iter_exec[j], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    AMG_HIP(e);
  }
  h->graphs_ready = true;
  return AMG_OK;
}

// Reduction scratch supplied by the caller of solve_impl (the no-allocation
// form); null members: the hierarchy's own buffers.
struct SolveScratch {
  double* scal = nullptr;
  double* partials = nullptr;
  unsigned* counter = nullptr;
};

// sx given (the no-allocation form): reductions use sx's buffers, and the
// solve captures no graphs, creates no events and queues no iteration ahead
// of the stopping test (one stream synchronization per outer iteration).
template <typename VT, typename MT>
int32_t solve_impl(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info,
                   const SolveScratch* sx = nullptr) {
  auto t0 = clk::now();
  Engine<VT, MT> E{h, s};
  const bool noalloc = sx != nullptr;
  if (noalloc) {
    E.scal_ = sx->scal;
    E.partials_ = sx->partials;
    E.counter_ = sx->counter;
    // the arrival counter must start at zero (a fill kernel, no memset node)
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, E.counter_);
    AMG_HIP(hipGetLastError());
  }
  double* const dscal = E.sc();
  const bool energy = h->p.stop == AMG_STOP_ENERGY;
  AMG_TRY(E.residual64(f, u, h->r, S_RR0));
  if (energy) {
    AMG_TRY(E.dot64(f, f, S_FF));
    AMG_TRY(E.energy64(u));
    AMG_HIP(hipMemcpyAsync(h->host_scal + 3, dscal + S_FF, sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(h->host_scal + 4, dscal + S_XR, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  AMG_HIP(hipMemcpyAsync(h->host_scal, dscal + S_RR0, sizeof(double), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const double rho0 = std::sqrt(h->host_scal[0]);
  // energy test: ||u_k||_A = sqrt((u_k, A u_k)) against ||u_0||_A
  const double en0 = energy ? std::sqrt(std::max(h->host_scal[4], 0.0)) : 0.0;
  if (energy && h->host_scal[3] != 0.0) {
    set_last_error("the A-norm error test solves A u = 0: f must be zero");
    return AMG_ERR_ARG;
  }
  const double ref0 = energy ? en0 : rho0;
  int32_t status = AMG_OK;
  int it = 0, test_it = 0, replaced = 0;
  double rel = ref0 > 0.0 ? 1.0 : 0.0;
  bool true_known = false;  // scal[S_RRT] holds ||f - A u||^2 of the returned u
  if (ref0 > 0.0) {
    const bool use_graph = h->p.use_graph != 0 && !noalloc;
    if (use_graph && (!h->graphs_ready || h->graph_u != u)) {
      AMG_TRY(capture_graphs<VT, MT>(h, u));
      h->graph_u = u;
    }
    if (!noalloc)
      for (hipEvent_t& e : h->iter_ev)
        if (!e) AMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const int R = h->p.restart;
    int pos_of[2] = {0, 0};  // window position of iteration k at [k & 1]
    int next_pos = 0;
    auto launch = [&](int k) -> int32_t {
      const int j = next_pos;
      pos_of[k & 1] = j;
      next_pos = j + 1 == R ? 0 : j + 1;
      if (use_graph) {
        AMG_HIP(hipGraphLaunch(h->iter_exec[j], s));
      } else {
        AMG_TRY(E.outer_iter(j, u));
      }
      if (!noalloc) AMG_HIP(hipEventRecord(h->iter_ev[k & 1], s));
      return AMG_OK;
    };
    // completion of iteration k (the no-allocation form has at most one
    // iteration in flight: the stream itself)
    auto wait = [&](int k) -> int32_t {
      if (noalloc) {
        AMG_HIP(hipStreamSynchronize(s));
      } else {
        AMG_HIP(hipEventSynchronize(h->iter_ev[k & 1]));
      }
      return AMG_OK;
    };
    auto pub = [&](int k) { return h->host_scal + kPubBase + 2 * pos_of[k & 1]; };
    auto ratio = [&](int k) {
      const double rr = pub(k)[0];
      return energy ? std::sqrt(std::max(rr, 0.0)) / en0 : std::sqrt(rr) / rho0;
    };
    auto broke = [&](int k) {
      const double rho = pub(k)[1];
      return !(rho > 0.0) || !std::isfinite(rho);
    };
    // Iteration k + 1 is queued before the test of iteration k is read when
    // the ratio predicted for k (the last one times the last reduction) is
    // above kAheadFactor x tol, so that the device does not idle while the
    // host reads; if the test passes at k after all, the queued iteration
    // still runs and is counted (test_iter keeps k).  (With a window of one
    // position both would publish into the same slot.)
    // A pass of the recursive residual test is confirmed on the true residual
    // r = f - A u, which replaces the recursive one; if it is still above
    // tol, the window restarts from it.
    status = AMG_ERR_MAXIT;
    AMG_TRY(launch(1));
    int queued = 1;
    double last = 1.0, before = 1.0;  // ratios of iterations k - 1 and k - 2
    for (it = 1; it <= h->p.max_iter; ++it) {
      const double predicted = last * std::min(1.0, last / before);
      if (!noalloc && R >= 2 && it >= 2 && queued == it && it < h->p.max_iter &&
          predicted > kAheadFactor * h->p.tol) {
        AMG_TRY(launch(it + 1));
        queued = it + 1;
      }
      AMG_TRY(wait(it));
      if (broke(it)) {
        status = AMG_ERR_BREAKDOWN;
        break;
      }
      rel = ratio(it);
      if (rel <= h->p.tol) {
        test_it = it;
        if (queued > it) {
          // the iteration queued ahead ran too: its update is in u
          AMG_TRY(wait(queued));
          it = queued;
          if (broke(it)) {
            status = AMG_ERR_BREAKDOWN;
            break;
          }
          rel = ratio(it);
        }
        if (energy) {
          status = AMG_OK;
          break;
        }
        AMG_TRY(E.residual64(f, u, h->r, S_RRT));
        AMG_HIP(hipMemcpyAsync(h->host_scal + 2, dscal + S_RRT, sizeof(double), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        true_known = true;
        const double rt = std::sqrt(h->host_scal[2]) / rho0;
        if (rt <= h->p.tol) {
          status = AMG_OK;
          break;
        }
        // restart from the true residual
        true_known = false;
        rel = rt;
        ++replaced;
        next_pos = 0;
        last = before = 1.0;
        if (it < h->p.max_iter) {
          AMG_TRY(launch(it + 1));
          queued = it + 1;
        }
        continue;
      }
      before = last;
      last = rel;
      if (queued == it && it < h->p.max_iter) {
        AMG_TRY(launch(it + 1));
        queued = it + 1;
      }
    }
    if (it > h->p.max_iter) it = h->p.max_iter;
    if (queued > it) {
      // an iteration queued ahead of a failing test ran too: report it
      AMG_TRY(wait(queued));
      it = queued;
      true_known = false;
    }
  }
  if (!true_known) {
    // true FP64 residual of the returned u
    AMG_TRY(E.residual64(f, u, h->tmp, S_RRT));
    AMG_HIP(hipMemcpyAsync(h->host_scal + 2, dscal + S_RRT, sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
  }
  if (info) {
    info->status = status;
    info->iters = it;
    info->rel_res = rel;
    info->rel_res_true = rho0 > 0.0 ? std::sqrt(h->host_scal[2]) / rho0 : 0.0;
    info->solve_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    info->test_iter = status == AMG_OK ? test_it : it;
    info->replacements = replaced;
  }
  return status;
}

// Record the tail program (the inner solve of the tail level and everything
// below it), place the data it touches in LDS, and upload it.  The tail level
// is the finest level t >= 1 with at most tail_rows rows whose levels t..L fit
// in the LDS left over by the kernel's static arrays.
// `g` names the buffer (the device array it mirrors); a constant buffer is
// copied in from `host` when given, else from `g`.
struct LdsBuf {
  const void* g;
  size_t bytes;
  bool copy_in;
  const void* host = nullptr;
};

inline size_t round16(size_t b) { return (b + 15) & ~size_t(15); }

// A tail level's matrix in the uniform-width layout the tail program reads
// (OffTail): the level's plain layout (64-row slices, rows in order) with
// every slice padded to the widest, rounded up to a multiple of 4, by zero
// weights on the row's own column.
struct TailMatHost {
  int pw = -1;
  std::vector<int> col;
  std::vector<char> val;
};

template <typename MT>
int32_t tail_mat_host(const Level& lv, hipStream_t s, TailMatHost& out) {
  const int ns = lv.plain_nslices;
  const Mat<MT> A = plain_mat_of<MT>(lv);
  std::vector<int> w(ns), off(ns + 1), col((size_t)lv.plain_entries);
  std::vector<MT> val((size_t)lv.plain_entries);
  AMG_HIP(hipMemcpyAsync(w.data(), A.width, sizeof(int) * ns, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipMemcpyAsync(off.data(), A.off, sizeof(int) * (ns + 1), hipMemcpyDeviceToHost, s));
  if (!col.empty()) {
    AMG_HIP(hipMemcpyAsync(col.data(), A.col, sizeof(int) * col.size(), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(val.data(), A.val, sizeof(MT) * val.size(), hipMemcpyDeviceToHost, s));
  }
  AMG_HIP(hipStreamSynchronize(s));
  int mw = 0;
  for (int x : w) mw = std::max(mw, x);
  const int pw = (mw + 3) & ~3;
  const size_t ent = (size_t)ns * pw * 64;
  out.pw = pw;
  out.col.assign(ent, 0);
  out.val.assign(sizeof(MT) * ent, 0);
  MT* pv = reinterpret_cast<MT*>(out.val.data());
  for (int sl = 0; sl < ns; ++sl)
    for (int p = 0; p < 64; ++p) {
      const int r = sl * 64 + p;
      const int self = r < lv.n ? r : 0;
      for (int t = 0; t < pw; ++t) {
        const size_t i = ((size_t)sl * pw + t) * 64 + p;
        const bool real = t < w[sl];
        out.col[i] = real ? col[(size_t)off[sl] + (size_t)t * 64 + p] : self;
        pv[i] = real ? val[(size_t)off[sl] + (size_t)t * 64 + p] : MT(0);
      }
    }
  return AMG_OK;
}

template <typename VT, typename MT>
void tail_buffers(const amg_hier* h, int t, const std::vector<TailMatHost>& mats, std::vector<LdsBuf>& bufs) {
  const size_t vt = sizeof(VT), mt = sizeof(MT);
  const int nu = h->p.inner_steps;
  for (int l = t; l < h->L; ++l) {
    const Level& lv = h->lv[l];
    const size_t n = lv.n;
    const Mat<MT> A = plain_mat_of<MT>(lv);
    const TailMatHost& M = mats[l];
    bufs.push_back({A.col, sizeof(int) * M.col.size(), true, M.col.data()});
    bufs.push_back({A.val, M.val.size(), true, M.val.data()});
    bufs.push_back({A.D, mt * n, true});
    bufs.push_back({lv.agg, sizeof(int) * n, true});
    bufs.push_back({lv.members, sizeof(int) * n, true});
    bufs.push_back({lv.member_off, sizeof(int) * (h->lv[l + 1].n + 1), true});
    const auto& W = h->ws[l];
    bufs.push_back({W.A, vt * n, false});
    bufs.push_back({W.B, vt * n, false});
    bufs.push_back({W.S, vt * n, false});
    bufs.push_back({W.rhs, vt * n, l == t});
    bufs.push_back({W.sol, vt * n, false});
    for (int k = 0; k < nu; ++k) {
      bufs.push_back({W.Z[k], vt * n, false});
      bufs.push_back({W.Q[k], vt * n, false});
    }
  }
  const size_t nL = h->nL;
  bufs.push_back({h->ws[h->L].rhs, vt * nL, false});
  bufs.push_back({h->ws[h->L].sol, vt * nL, false});
  bufs.push_back({h->chol_inv, sizeof(double) * nL * nL, true});
  bufs.push_back({h->chol_invT, sizeof(double) * nL * nL, true});
  bufs.push_back({h->scal, sizeof(double) * SCAL_SIZE, false});
}

// Words of the auxiliary area an op needs (operand lists of inner products
// and direction updates).
inline size_t aux_words(const TailOp& o) {
  if (o.type == OP_MULTIDOT) return 2 * (size_t)o.k;
  if (o.type == OP_FCG_P) return 3 * (size_t)o.k;
  return 0;
}

// Auxiliary words of all ops, each op's list starting on 16 bytes.
inline size_t aux_total(const std::vector<TailOp>& ops) {
  size_t aux = 0;
  for (const auto& o : ops) aux += (aux_words(o) + 3) & ~size_t(3);
  return aux;
}

// Instructions are kept in device memory; the LDS image starts with the
// auxiliary operand lists.
inline size_t header_bytes(const std::vector<TailOp>& ops) { return round16(aux_total(ops) * sizeof(int32_t)); }

template <typename VT, typename MT>
int32_t prepare_tail(amg_hier* h, hipStream_t s) {
  h->tail_level = 0;
  if (h->p.tail_rows <= 0 || h->L < 2 || !h->chol_inv) return AMG_OK;
  int max_lds = 0;
  AMG_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
  const size_t static_lds = sizeof(double) * (16 * 8 + 2 * 1024) + 1024;  // red, sb, sy + margin
  if ((size_t)max_lds <= static_lds) return AMG_OK;
  const size_t budget = (size_t)max_lds - static_lds;
  // LDS image: [auxiliary operand lists][level data ...]
  int t = 0;
  std::vector<TailMatHost> mats(h->L);
  for (int cand = h->L - 1; cand >= 1; --cand) {
    if (h->lv[cand].n > h->p.tail_rows || h->lv[cand].n > kTailMaxRows || !h->lv[cand].plain_off) break;
    AMG_TRY(tail_mat_host<MT>(h->lv[cand], s, mats[cand]));
    std::vector<LdsBuf> bufs;
    tail_buffers<VT, MT>(h, cand, mats, bufs);
    std::vector<TailOp> ops;
    {
      Engine<VT, MT> E{h, s, &ops};
      if (E.coarse_correction(cand) != AMG_OK) break;
    }
    size_t tot = header_bytes(ops);
    for (const auto& b : bufs) tot += round16(b.bytes);
    if (tot > budget) break;
    t = cand;
  }
  if (t == 0) return AMG_OK;
  std::vector<TailOp> ops;
  {
    Engine<VT, MT> E{h, s, &ops};
    AMG_TRY(E.coarse_correction(t));
  }
  // the last step, sol += alpha p on the tail level, goes into the copy-out
  TailOp fin{};
  const bool fold_fin = !ops.empty() && ops.back().type == OP_FCG_XR && ops.back().i2 == 0 && ops.back().i3 == 0 &&
                        ops.back().c == h->ws[t].sol;
  if (fold_fin) {
    fin = ops.back();
    ops.pop_back();
  }
  const uint32_t aux_off = 0;
  uint64_t off = header_bytes(ops);
  std::vector<LdsBuf> bufs;
  tail_buffers<VT, MT>(h, t, mats, bufs);
  // image order: the header, then every constant buffer (one contiguous
  // region, copied in from one packed device blob), then the tail level's
  // right-hand side (the only per-call input), then the work vectors
  const void* rhs_t = h->ws[t].rhs;
  std::stable_partition(bufs.begin(), bufs.end(), [&](const LdsBuf& b) { return b.copy_in && b.g != rhs_t; });
  std::stable_partition(bufs.begin(), bufs.end(), [&](const LdsBuf& b) { return b.copy_in; });
  std::vector<std::pair<const void*, uint64_t>> map;
  std::vector<std::pair<const LdsBuf*, uint64_t>> consts;
  uint64_t rhs_off = 0, rhs_bytes = 0, const_end = 0;
  for (const auto& b : bufs) {
    map.push_back({b.g, off});
    if (b.copy_in && b.g != rhs_t) {
      consts.push_back({&b, off});
      const_end = off + round16(b.bytes);
    } else if (b.g == rhs_t) {
      rhs_off = off;
      rhs_bytes = round16(b.bytes);
    }
    off += round16(b.bytes);
  }
  const size_t need = off;
  // every operand of the program must be one of the placed buffers
  bool ok = true;
  auto lo = [&](const void* p) -> uint32_t {
    if (!p) return 0;
    for (const auto& m : map)
      if (m.first == p) return (uint32_t)m.second;
    ok = false;
    return 0;
  };
  std::vector<TailInstr> ins(ops.size());
  std::vector<int32_t> aux;
  for (size_t i = 0; i < ops.size(); ++i) {
    const TailOp& o = ops[i];
    TailInstr& I = ins[i];
    std::memset(&I, 0, sizeof(I));
    I.type = o.type;
    I.n = o.n;
    I.k = o.k;
    I.i0 = o.i0;
    I.i1 = o.i1;
    I.i2 = o.i2;
    I.i3 = o.i3;
    I.f0 = o.f0;
    I.f1 = o.f1;
    I.f2 = o.f2;
    I.f3 = o.f3;
    I.a = lo(o.a);
    I.b = lo(o.b);
    I.c = lo(o.c);
    I.d = lo(o.d);
    if (o.level >= t && o.level < h->L) {
      const Mat<MT> A = plain_mat_of<MT>(h->lv[o.level]);
      const Transfer T = transfer_of(h, o.level);
      switch (o.type) {
        case OP_CHEB_FIRST: case OP_CHEB_NEXT: case OP_RESIDUAL: case OP_RESIDUAL_P: case OP_SPMV_DOTS:
          I.off = 0;
          I.width = (uint32_t)mats[o.level].pw;
          I.col = lo(A.col);
          I.val = lo(A.val);
          I.D = lo(A.D);
          break;
        default:
          break;
      }
      if (o.type == OP_RESTRICT) {
        I.members = lo(T.members);
        I.member_off = lo(T.member_off);
      }
      if (o.type == OP_PROLONG || o.type == OP_RESIDUAL_P || (o.type == OP_CHEB_FIRST && o.i2)) I.agg = lo(T.agg);
    }
    if (o.type == OP_RESIDUAL_P || (o.type == OP_CHEB_FIRST && o.i2)) I.e = lo(o.w.p[0]);
    if (o.type == OP_SPMV_DOTS) {
      I.i0 = o.s0.s[0];
      I.i1 = o.s0.s[1];
    }
    if (o.k == 1 && (o.type == OP_MULTIDOT || o.type == OP_FCG_P)) {
      I.b = lo(o.w.p[0]);
      I.i0 = o.s0.s[0];
      I.i1 = o.type == OP_FCG_P ? o.s1.s[0] : 0;
    }
    if (aux_words(o)) {
      I.aux = aux_off + (uint32_t)(aux.size() * sizeof(int32_t));
      for (int j = 0; j < o.k; ++j) aux.push_back((int32_t)lo(o.w.p[j]));
      for (int j = 0; j < o.k; ++j) aux.push_back(o.s0.s[j]);
      if (o.type == OP_FCG_P)
        for (int j = 0; j < o.k; ++j) aux.push_back(o.s1.s[j]);
      while (aux.size() & 3) aux.push_back(0);
    }
  }
  const uint32_t linv = lo(h->chol_inv);
  const uint32_t linvt = lo(h->chol_invT);
  const uint32_t scal_t = lo(h->scal);
  const uint32_t sol_t = lo(h->ws[t].sol);
  if (!ok || need > budget) {
    set_last_error("tail program refers to data outside its LDS image");
    return AMG_ERR_DEVICE;
  }
  // the header (operand lists) and the constant buffers packed into one
  // device blob laid out as the start of the LDS image; the instructions
  // follow it in device memory (read from there, not copied into LDS)
  std::vector<char> head(header_bytes(ops), 0);
  if (!aux.empty()) std::memcpy(head.data() + aux_off, aux.data(), aux.size() * sizeof(int32_t));
  const size_t blob_bytes = std::max<size_t>(head.size(), const_end);
  const size_t code_at = ((blob_bytes + 63) & ~size_t(63)) + 256;  // instructions on 64-byte lines
  char* d_blob = nullptr;
  void* d_cin = nullptr;
  AMG_TRY(dalloc(h, (void**)&d_blob, code_at + ins.size() * sizeof(TailInstr) + 16));
  if (!head.empty()) AMG_HIP(hipMemcpyAsync(d_blob, head.data(), head.size(), hipMemcpyHostToDevice, s));
  AMG_HIP(hipMemcpyAsync(d_blob + code_at, ins.data(), ins.size() * sizeof(TailInstr), hipMemcpyHostToDevice, s));
  for (const auto& c : consts)
    if (c.first->bytes > 0)
      AMG_HIP(hipMemcpyAsync(d_blob + c.second, c.first->host ? c.first->host : c.first->g, c.first->bytes,
                             c.first->host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
  std::vector<TailCopy> cin;
  cin.push_back(TailCopy{d_blob, 0, (int)round16(blob_bytes)});
  if (rhs_bytes) cin.push_back(TailCopy{rhs_t, (uint32_t)rhs_off, (int)rhs_bytes});
  AMG_TRY(dalloc(h, &d_cin, cin.size() * sizeof(TailCopy) + 16));
  AMG_HIP(hipMemcpyAsync(d_cin, cin.data(), cin.size() * sizeof(TailCopy), hipMemcpyHostToDevice, s));
  AMG_HIP(hipStreamSynchronize(s));
  TailProgram P;
  std::memset(&P, 0, sizeof(P));
  P.nops = (int)ops.size();
  P.ncin = (int)cin.size();
  P.ops = reinterpret_cast<const TailInstr*>(d_blob + code_at);
  P.scal_off = scal_t;
  P.cin = (const TailCopy*)d_cin;
  P.cout = TailCopy{h->ws[t].sol, sol_t, (int)round16(sizeof(VT) * h->lv[t].n)};
  P.linv_off = linv;
  P.linvt_off = linvt;
  P.nL = h->nL;
  if (fold_fin) {
    P.fin_p = lo(fin.a);
    P.fin_rho = fin.i0;
    P.fin_gam = fin.i1;
    P.fin_n = h->lv[t].n;
    if (!ok || P.fin_p == 0) {
      set_last_error("tail program: the folded last step refers to data outside its LDS image");
      return AMG_ERR_DEVICE;
    }
  }
  h->tail_prog_storage.resize(sizeof(TailProgram));
  std::memcpy(h->tail_prog_storage.data(), &P, sizeof(P));
  h->tail_prog = h->tail_prog_storage.data();
  h->tail_lds_bytes = need;
  h->tail_threads = std::min(TAIL_THREADS, std::max(64, (h->lv[t].n + 63) / 64 * 64));
  (void)hipFuncSetAttribute((const void*)k_tail<VT, MT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
  h->tail_nops = P.nops;
  h->tail_level = t;
  return AMG_OK;
}

}  // namespace

void destroy_graphs(amg_hier* h) {
  for (int j = 0; j < 8; ++j) {
    if (h->iter_exec[j]) (void)hipGraphExecDestroy(h->iter_exec[j]);
    h->iter_exec[j] = nullptr;
  }
  for (hipEvent_t& e : h->iter_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  h->graphs_ready = false;
}

int32_t prepare_solve_impl(amg_hier* h, hipStream_t s);

// ---- stationary AMLI: the coarse-correction polynomials
constexpr int kAmliPowerIters = 20;
// a below 3 - 2 sqrt(2) would make the degree-1 polynomial negative near t = 1
constexpr double kAmliMinA = 0.18, kAmliMaxA = 0.99;

// g0 + g1 t: the degree-1 best uniform approximation to 1/t on [a, 1] (the
// smoother's closed form with lambda1 = 1, lambda0 = a).
void amli_poly(double a, double* g0, double* g1) {
  const double theta = 0.5 * (1.0 + a), eta = 0.5 * (1.0 - a);
  const double sk = std::sqrt(1.0 / a);
  const double dl = (sk - 1.0) / (sk + 1.0);
  const double om = 1.0 - dl * dl;
  const double c0 = 2.0 * dl / om;
  const double c1 = -4.0 * dl * dl / (om * om);
  *g1 = c1 / (eta * eta);
  *g0 = (c0 - c1 * theta / eta) / eta;
}

// lambda_min(B_l A_l) for l = L-1 .. 1 (each B_l uses the polynomials of the
// levels below it): power iteration on I - B_l A_l in the A_l inner product
// from a counter-based start vector, Rayleigh quotients mu, a_l = 1 - mu.
template <typename VT, typename MT>
int32_t estimate_amli(amg_hier* h, hipStream_t s) {
  const auto t0 = clk::now();
  const int L = h->L;
  h->amli_a.assign(L + 1, 0.0);
  h->amli_g0.assign(L + 1, 0.0);
  h->amli_g1.assign(L + 1, 0.0);
  Engine<VT, MT> E{h, s};
  std::vector<VT> v0;
  double sc[4];
  constexpr int S_VAV = S_DOTS, S_VV = S_DOTS + 1, S_WAW = S_DOTS + 2, S_WAV = S_DOTS + 3;
  for (int l = L - 1; l >= 1; --l) {
    const int n = h->lv[l].n;
    auto& W = h->ws[l];
    VT* V = static_cast<VT*>(W.Q[1]);
    VT* AV = static_cast<VT*>(W.Q[0]);
    VT* Y = static_cast<VT*>(W.Z[0]);
    VT* AW = static_cast<VT*>(W.Z[1]);
    if (!V || !AV || !Y || !AW) {
      set_last_error("AMLI needs the two-step workspace on every coarse level");
      return AMG_ERR_ARG;
    }
    v0.resize(n);
    const uint64_t base = (uint64_t)l << 40;
    for (int i = 0; i < n; ++i)
      v0[i] = (VT)(2.0 * ((double)(splitmix64(base + (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0);
    AMG_HIP(hipMemcpyAsync(V, v0.data(), sizeof(VT) * n, hipMemcpyHostToDevice, s));
    double mu = 0.0;
    for (int it = 0; it < kAmliPowerIters; ++it) {
      AMG_TRY(E.spmv_dots(l, V, AV, V, slots2(S_VAV, S_VV)));
      AMG_TRY(E.kcycle(l, static_cast<const VT*>(AV), Y));
      hipLaunchKernelGGL((k_axpby<VT>), dim3(nblk(n)), dim3(TPB), 0, s, n, 1.0, (const VT*)V, -1.0, (const VT*)Y, Y);
      AMG_HIP(hipGetLastError());
      AMG_TRY(E.spmv_dots(l, Y, AW, AV, slots2(S_WAW, S_WAV)));
      AMG_HIP(hipMemcpyAsync(sc, h->scal + S_DOTS, sizeof(sc), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      mu = sc[3] / sc[0];
      const double ww = sc[2];
      if (!(ww > 0.0) || !std::isfinite(ww)) break;
      hipLaunchKernelGGL((k_axpby<VT>), dim3(nblk(n)), dim3(TPB), 0, s, n, 1.0 / std::sqrt(ww), (const VT*)Y, 0.0,
                         (const VT*)V, V);
      AMG_HIP(hipGetLastError());
    }
    const double a = std::min(std::max(1.0 - mu, kAmliMinA), kAmliMaxA);
    h->amli_a[l] = a;
    amli_poly(a, &h->amli_g0[l], &h->amli_g1[l]);
    h->desc.amli_lambda_min[l] = a;
  }
  AMG_HIP(hipStreamSynchronize(s));
  h->desc.setup_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  return AMG_OK;
}

// The aggregate-to-block map of the fused residual + restriction on level l:
// aggregates in order, packed greedily into blocks of at most TPB member
// rows; members must be listed aggregate by aggregate.  Sorted layouts also
// get the row-to-slot map.  Levels where a single aggregate exceeds a block
// keep the two separate steps.
int32_t prepare_restrict_residual(amg_hier* h, int l, hipStream_t s) {
  const Level& lv = h->lv[l];
  const int n = lv.n, nc = h->lv[l + 1].n;
  std::vector<int> moff(nc + 1);
  AMG_HIP(hipMemcpyAsync(moff.data(), lv.member_off, sizeof(int) * (nc + 1), hipMemcpyDeviceToHost, s));
  std::vector<int> perm;
  if (lv.sell_perm) {
    perm.resize(n);
    AMG_HIP(hipMemcpyAsync(perm.data(), lv.sell_perm, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  }
  AMG_HIP(hipStreamSynchronize(s));
  if (moff[0] != 0 || moff[nc] != n) return AMG_OK;
  std::vector<int> blk{0};
  int rows = 0;
  for (int J = 0; J < nc; ++J) {
    const int sz = moff[J + 1] - moff[J];
    if (sz > TPB) return AMG_OK;
    if (rows + sz > TPB) {
      blk.push_back(J);
      rows = 0;
    }
    rows += sz;
  }
  blk.push_back(nc);
  auto& W = h->ws[l];
  AMG_TRY(dalloc(h, &W.agg_blk, sizeof(int) * blk.size()));
  AMG_HIP(hipMemcpyAsync(W.agg_blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice, s));
  W.n_agg_blk = (int)blk.size() - 1;
  if (lv.sell_perm) {
    std::vector<int> inv(n);
    for (int q = 0; q < n; ++q) inv[perm[q]] = q;
    AMG_TRY(dalloc(h, &W.slot_of_row, sizeof(int) * n));
    AMG_HIP(hipMemcpyAsync(W.slot_of_row, inv.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  }
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

int32_t prepare_solve(amg_hier* h, hipStream_t s) {
  const size_t before = h->bytes;
  const int32_t st = prepare_solve_impl(h, s);
  h->ws_bytes = h->bytes - before;
  return st;
}

int32_t prepare_solve_impl(amg_hier* h, hipStream_t s) {
  for (int l = 0; l < std::max(h->L, 1); ++l) {
    const Level& lv = h->lv[l];
    if (!lv.sell_off || !lv.sell_w || !lv.sell_col || !lv.sell_val || !lv.D ||
        (h->mixed && (!lv.sell_valf || !lv.Df))) {
      set_last_error("level " + std::to_string(l) + " has no sliced-ELL form");
      return AMG_ERR_DEVICE;
    }
  }
  const size_t vt = h->mixed ? sizeof(float) : sizeof(double);
  h->ws.assign(h->lv.size(), amg_hier::Work{});
  for (int l = 0; l <= h->L; ++l) {
    const size_t n = h->lv[l].n;
    auto& W = h->ws[l];
    if (l < h->L) {
      AMG_TRY(dalloc(h, &W.A, n * vt + 16));
      AMG_TRY(dalloc(h, &W.B, n * vt + 16));
      AMG_TRY(dalloc(h, &W.S, n * vt + 16));
    }
    if (l >= 1) {
      AMG_TRY(dalloc(h, &W.rhs, n * vt + 16));
      AMG_TRY(dalloc(h, &W.sol, n * vt + 16));
    }
    if (l >= 1 && l < h->L) {
      for (int k = 0; k < h->p.inner_steps; ++k) {
        AMG_TRY(dalloc(h, &W.Z[k], n * vt + 16));
        AMG_TRY(dalloc(h, &W.Q[k], n * vt + 16));
      }
      if (h->p.fuse && h->p.inner_steps == 2 && h->p.degree > 0 && n < (size_t)kFoldProlongRows) {
        AMG_TRY(dalloc(h, &W.rhs2, n * vt + 16));
        AMG_TRY(dalloc(h, &W.P1, n * vt + 16));
      }
    }
    if (h->p.fuse && l < h->L && n < (size_t)kFoldProlongRows) AMG_TRY(prepare_restrict_residual(h, l, s));
  }
  const size_t n0 = h->lv[0].n;
  AMG_TRY(dalloc(h, &h->r, n0));
  AMG_TRY(dalloc(h, &h->tmp, n0));
  AMG_TRY(dalloc(h, &h->z, n0 * vt + 16));
  for (int j = 0; j < h->p.restart; ++j) {
    AMG_TRY(dalloc(h, &h->P[j], n0));
    AMG_TRY(dalloc(h, &h->Qo[j], n0));
  }
  h->max_blocks = nblk(n0);
  // grids of up to this many blocks finish their reductions in-kernel (one
  // release fence per block); larger grids use the one-block finishing kernel
  h->last_block_max = 32;
  if (const char* e = std::getenv("AMG_LAST_BLOCK_MAX")) h->last_block_max = std::max(0, std::atoi(e));
  AMG_TRY(dalloc(h, &h->partials, (size_t)std::max(h->max_blocks, 1) * 8));
  AMG_TRY(dalloc(h, &h->scal, SCAL_SIZE));
  AMG_TRY(dalloc(h, &h->counter, 1));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, h->counter);
  AMG_HIP(hipGetLastError());
  // the single-system solve's pinned mirror of its stopping test (workspace
  // clones serve batches, which keep their state on the device)
  if (!h->parent) AMG_HIP(hipHostMalloc((void**)&h->host_scal, 64 * sizeof(double), hipHostMallocCoherent));
  AMG_HIP(hipStreamSynchronize(s));
  if (h->p.cycle == AMG_CYCLE_AMLI && h->amli_g0.empty()) {
    // the cycle on each level runs through device-wide kernels here: the tail
    // program (which records these polynomials) is prepared afterwards
    if (h->mixed) {
      AMG_TRY(estimate_amli<float, float>(h, s));
    } else {
      AMG_TRY(estimate_amli<double, double>(h, s));
    }
  }
  if (h->mixed) {
    AMG_TRY(prepare_tail<float, float>(h, s));
  } else {
    AMG_TRY(prepare_tail<double, double>(h, s));
  }
  return AMG_OK;
}

int32_t solve(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info) {
  if (h->mixed) return solve_impl<float, float>(h, f, u, s, info);
  return solve_impl<double, double>(h, f, u, s, info);
}

// ---- the no-allocation solve
// Its reduction scratch (scalar area, arrival counter, block partials) is this
// array: one copy per device, held until the process ends, shared by every
// no-allocation solve on that device.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address): it
// uses the address hipGetSymbolAddress returns for the current device.
namespace {
constexpr size_t kScratchScalBytes = (sizeof(double) * SCAL_SIZE + 255) / 256 * 256;
constexpr size_t kScratchCounterBytes = 256;
constexpr size_t kScratchPartialsOff = kScratchScalBytes + kScratchCounterBytes;
static_assert(kScratchPartialsOff < kNoAllocScratchBytes, "scratch layout");
// reduction partials: 8 doubles per block of the finest level
constexpr size_t kScratchMaxBlocks = (kNoAllocScratchBytes - kScratchPartialsOff) / (8 * sizeof(double));
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (which is current), looked up
// once per device.
int32_t scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("device index out of range for the no-allocation scratch");
    return AMG_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    AMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
      set_last_error("hipGetSymbolAddress returned a null scratch address");
      return AMG_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return AMG_OK;
}
}  // namespace

size_t noalloc_max_rows() { return kScratchMaxBlocks * (size_t)TPB; }

int32_t solve_noalloc(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info) {
  if ((size_t)std::max(h->max_blocks, 1) > kScratchMaxBlocks) {
    set_last_error("amg_solve_noalloc: the finest level has " + std::to_string(h->lv[0].n) +
                   " rows; its reduction scratch holds at most " + std::to_string(noalloc_max_rows()) + " rows");
    return AMG_ERR_ARG;
  }
  int dev = -1;
  AMG_HIP(hipGetDevice(&dev));
  if (dev != h->device) {
    set_last_error("amg_solve_noalloc: the hierarchy lives on device " + std::to_string(h->device) +
                   ", the current device is " + std::to_string(dev));
    return AMG_ERR_ARG;
  }
  unsigned char* base = nullptr;
  AMG_TRY(scratch_address(dev, &base));
  SolveScratch sx;
  sx.scal = reinterpret_cast<double*>(base);
  sx.counter = reinterpret_cast<unsigned*>(base + kScratchScalBytes);
  sx.partials = reinterpret_cast<double*>(base + kScratchPartialsOff);
  if (h->mixed) return solve_impl<float, float>(h, f, u, s, info, &sx);
  return solve_impl<double, double>(h, f, u, s, info, &sx);
}

template <typename VT>
int32_t time_layout_impl(const Level& lv, void* wk, void* wb, void* y, hipStream_t s, float* ms) {
  const Mat<VT> A = mat_of<VT>(lv);
  const dim3 grid(A.nb), block(TPB << A.lk);
  auto launch = [&]() {
    hipLaunchKernelGGL((k_cheb_next<VT, VT, VT, true, kStepCoarse>), grid, block, 0, s, A, (const VT*)wk, (const VT*)wb,
                       (VT*)wb, (VT*)y, lv.theta, lv.eta > 0.0 ? 2.0 / lv.eta : 1.0, 1e-3);
  };
  launch();
  launch();
  AMG_HIP(hipGetLastError());
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  constexpr int kReps = 5;
  float best = 0.f;
  hipError_t e = hipSuccess;
  for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
    e = hipEventRecord(e0, s);
    for (int i = 0; i < kReps; ++i) launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (trial == 0 || t < best) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  AMG_HIP(e);
  *ms = best / kReps;
  return AMG_OK;
}

int32_t time_cheb_layout(const Level& lv, bool mixed, void* wk, void* wb, void* y, hipStream_t s, float* ms) {
  return mixed ? time_layout_impl<float>(lv, wk, wb, y, s, ms) : time_layout_impl<double>(lv, wk, wb, y, s, ms);
}

int32_t time_step(amg_hier* h, int reps, hipStream_t s, amg_kernel_timing* t) {
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  int32_t st;
  if (h->mixed) {
    Engine<float, float> E{h, s};
    st = E.time_fine_step(reps, e0, e1);
  } else {
    Engine<double, double> E{h, s};
    st = E.time_fine_step(reps, e0, e1);
  }
  float ms = 0.f;
  if (st == AMG_OK) {
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      set_last_error(std::string("event timing: ") + hipGetErrorString(e));
      st = AMG_ERR_DEVICE;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::memset(t, 0, sizeof(*t));
  t->launches = reps;
  t->avg_ms = ms / reps;
  t->rows = h->lv[0].n;
  t->nnz = h->lv[0].nnz;
  t->entries = h->lv[0].sell_entries;
  t->grid = (int32_t)nblk(h->lv[0].n);
  t->value_bytes = h->mixed ? 4 : 8;
  return st;
}

// Rotating-copies timing of the finest level's storing Chebyshev step: copy 0
// is the level itself, copies 1 .. nc-1 are device copies of its column
// indices, weights, diagonal (and slot map) and of the step's three vectors.
template <typename VT, typename MT>
int32_t time_rotating_impl(amg_hier* h, int reps, int nc, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                           std::vector<void*>& owned) {
  const Level& lv = h->lv[0];
  const size_t n = lv.n, ent = lv.sell_entries;
  std::vector<Mat<MT>> mats(nc, mat_of<MT>(lv));
  std::vector<VT*> wk(nc), wb(nc), y(nc);
  wk[0] = static_cast<VT*>(h->ws[0].A);
  wb[0] = static_cast<VT*>(h->ws[0].B);
  y[0] = static_cast<VT*>(h->ws[0].S);
  auto dup = [&](const void* src, size_t bytes, void** dst) -> int32_t {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      set_last_error(std::string("hipMalloc (timing copies): ") + hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;
    }
    owned.push_back(p);
    AMG_HIP(hipMemcpyAsync(p, src, bytes, hipMemcpyDeviceToDevice, s));
    *dst = p;
    return AMG_OK;
  };
  for (int c = 1; c < nc; ++c) {
    void *col, *val, *D, *a, *b, *yy;
    AMG_TRY(dup(mats[0].col, ent * sizeof(int), &col));
    AMG_TRY(dup(mats[0].val, ent * sizeof(MT), &val));
    AMG_TRY(dup(mats[0].D, n * sizeof(MT), &D));
    AMG_TRY(dup(wk[0], n * sizeof(VT), &a));
    AMG_TRY(dup(wb[0], n * sizeof(VT), &b));
    AMG_TRY(dup(y[0], n * sizeof(VT), &yy));
    mats[c].col = static_cast<const int*>(col);
    mats[c].val = static_cast<const MT*>(val);
    mats[c].D = static_cast<const MT*>(D);
    if (mats[0].perm) {
      void* perm;
      AMG_TRY(dup(mats[0].perm, n * sizeof(int), &perm));
      mats[c].perm = static_cast<const int*>(perm);
    }
    wk[c] = static_cast<VT*>(a);
    wb[c] = static_cast<VT*>(b);
    y[c] = static_cast<VT*>(yy);
  }
  Engine<VT, MT> E{h, s};
  return E.time_fine_step_rotating(reps, nc, mats.data(), wk.data(), wb.data(), y.data(), e0, e1);
}

int32_t time_step_rotating(amg_hier* h, int reps, int copies, hipStream_t s, amg_kernel_timing* t) {
  hipEvent_t e0, e1;
  AMG_HIP(hipEventCreate(&e0));
  AMG_HIP(hipEventCreate(&e1));
  std::vector<void*> owned;
  int32_t st = h->mixed ? time_rotating_impl<float, float>(h, reps, copies, s, e0, e1, owned)
                        : time_rotating_impl<double, double>(h, reps, copies, s, e0, e1, owned);
  float ms = 0.f;
  if (st == AMG_OK) {
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      set_last_error(std::string("event timing: ") + hipGetErrorString(e));
      st = AMG_ERR_DEVICE;
    }
  }
  (void)hipStreamSynchronize(s);
  for (void* p : owned) (void)hipFree(p);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::memset(t, 0, sizeof(*t));
  t->launches = reps;
  t->avg_ms = ms / reps;
  t->rows = h->lv[0].n;
  t->nnz = h->lv[0].nnz;
  t->entries = h->lv[0].sell_entries;
  t->grid = (int32_t)nblk(h->lv[0].n);
  t->value_bytes = h->mixed ? 4 : 8;
  return st;
}

// ---- single steps (FP64 hierarchies, except the cycle) ------------------------
int32_t step_smoother(amg_hier* h, int l, const double* r, double* y, hipStream_t s) {
  Engine<double, double> E{h, s};
  return E.smooth(l, r, y, false);
}

int32_t step_residual(amg_hier* h, int l, const double* f, const double* x, double* out, hipStream_t s) {
  Engine<double, double> E{h, s};
  return E.residual(l, f, x, out);
}

int32_t step_restrict(amg_hier* h, int l, const double* sv, double* b, hipStream_t s) {
  Engine<double, double> E{h, s};
  return E.restrict_(l, sv, b);
}

int32_t step_prolong(amg_hier* h, int l, const double* e, double* x, hipStream_t s) {
  Engine<double, double> E{h, s};
  return E.prolong(l, e, x);
}

int32_t step_coarse(amg_hier* h, const double* b, double* x, hipStream_t s) {
  Engine<double, double> E{h, s};
  return E.coarse(b, x);
}

int32_t step_cycle(amg_hier* h, const double* r, double* z, hipStream_t s) {
  if (!h->mixed) {
    Engine<double, double> E{h, s};
    return E.kcycle(0, r, z);
  }
  Engine<float, float> E{h, s};
  float* zf = static_cast<float*>(h->z);
  AMG_TRY(E.kcycle(0, r, zf));
  const int n = h->lv[0].n;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(n)), dim3(TPB), 0, s, n, zf, z);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

}  // namespace amg
