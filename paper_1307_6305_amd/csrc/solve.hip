// Solve phase on the device: flexible CG preconditioned by the nonlinear AMLI
// cycle (k-cycle) with the best-uniform-approximation polynomial smoother
// (Sections 3 and 4 of the paper).
//
// Kernels (one row per lane over sliced ELL, slice height 64 = one wavefront):
//   k_cheb_first / k_cheb_next  one Chebyshev three-term step of q_m(A): SpMV,
//                               recurrence and the accumulation y += c_k w_k
//                               fused in one pass over the matrix
//   k_residual                  s = r - A x
//   k_restrict                  b = P^T s as a segmented sum over the member
//                               list of each aggregate (P is never stored)
//   k_prolong                   x += P e as a gather of the aggregate value
//   k_chol_solve_*              coarsest solve with the dense Cholesky factor
//   k_multidot, k_fcg_p,        flexible-CG steps; inner products are
//   k_spmv_dots, k_fcg_xr       deterministic fused grid reductions in FP64
//
// Scalars (inner products and the coefficients derived from them) never leave
// the device inside an iteration; the host reads two numbers per outer
// iteration for the stopping test.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "device_util.h"
#include "hier.h"

namespace amg {
namespace {

constexpr int TPB = 256;
constexpr int RED_BLOCKS = 1024;  // grid of the vector kernels with reductions

// Scalar area.  Outer iteration: rr, (p,q), (p,r), window dots, window rho.
// Inner solve on level l: base(l) + [0,8) rho_k, [8,16) gamma_k, [16,24) dots.
constexpr int S_RR = 0, S_RHO = 1, S_GAM = 2, S_RR0 = 3, S_RRT = 4, S_DUMMY = 7, S_DOTS = 8, S_RHOW = 16;
inline int lbase(int l) { return 64 + 32 * l; }
constexpr int SCAL_SIZE = 64 + 32 * (AMG_MAX_LEVELS + 1);

inline int nblk(int64_t n, int tpb = TPB) { return (int)std::max<int64_t>(1, (n + tpb - 1) / tpb); }
inline int rblk(int64_t n) { return std::min(RED_BLOCKS, nblk(n)); }

struct VecPtrs {
  const void* p[8];
};

template <typename MT>
struct Mat {
  int n;
  int nb;  // blocks of TPB rows
  const int* __restrict__ off;
  const int* __restrict__ width;
  const int* __restrict__ col;
  const MT* __restrict__ val;
  const MT* __restrict__ D;
};

template <typename MT>
Mat<MT> mat_of(const Level& lv);
template <>
Mat<double> mat_of<double>(const Level& lv) {
  return Mat<double>{lv.n, nblk(lv.n), lv.sell_off, lv.sell_w, lv.sell_col, lv.sell_val, lv.D};
}
template <>
Mat<float> mat_of<float>(const Level& lv) {
  return Mat<float>{lv.n, nblk(lv.n), lv.sell_off, lv.sell_w, lv.sell_col, lv.sell_valf, lv.Df};
}

// Row handled by this thread (XCD-aware tile order), or -1.
template <typename MT>
__device__ __forceinline__ int row_of(const Mat<MT>& A) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int r = tile * TPB + threadIdx.x;
  return r < A.n ? r : -1;
}

// sum_j W_rj x_j over the stored off-diagonal entries of row r.
template <typename AT, typename MT, typename XT>
__device__ __forceinline__ AT offdiag(const Mat<MT>& A, int r, const XT* __restrict__ x) {
  const int s = r >> 6, lane = r & 63;
  const int* __restrict__ c = A.col + A.off[s] + lane;
  const MT* __restrict__ v = A.val + A.off[s] + lane;
  const int wd = A.width[s];
  AT acc = 0;
#pragma unroll 4
  for (int k = 0; k < wd; ++k) acc += (AT)v[k * kWave] * (AT)x[c[k * kWave]];
  return acc;
}

// ------------------------------------------------------------------ smoother
// w1 = (A w0 - theta w0) / eta;  y = [y +] c0 w0 + c1 w1   (c already / eta)
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(TPB) k_cheb_first(Mat<MT> A, const RT* __restrict__ w0, VT* __restrict__ w1,
                                                    VT* __restrict__ y, double theta, double inv_eta, double c0,
                                                    double c1, int accum, int store) {
  using AT = VT;
  const int r = row_of(A);
  if (r < 0) return;
  const AT x0 = (AT)w0[r];
  const AT ax = (AT)A.D[r] * x0 - offdiag<AT>(A, r, w0);
  const AT t = (ax - (AT)theta * x0) * (AT)inv_eta;
  if (store) w1[r] = (VT)t;
  AT yy = (AT)c0 * x0 + (AT)c1 * t;
  if (accum) yy += (AT)y[r];
  y[r] = (VT)yy;
}

// w_{k+1} = 2 (A w_k - theta w_k) / eta - w_{k-1};  y += c_{k+1} w_{k+1}.
// wnext may alias wprev (each element is read before it is overwritten).
template <typename VT, typename MT, typename PT>
__global__ void __launch_bounds__(TPB) k_cheb_next(Mat<MT> A, const VT* __restrict__ wk, const PT* wprev, VT* wnext,
                                                   VT* __restrict__ y, double theta, double two_inv_eta, double ck,
                                                   int store) {
  using AT = VT;
  const int r = row_of(A);
  if (r < 0) return;
  const AT xk = (AT)wk[r];
  const AT ax = (AT)A.D[r] * xk - offdiag<AT>(A, r, wk);
  const AT t = (ax - (AT)theta * xk) * (AT)two_inv_eta - (AT)wprev[r];
  if (store) wnext[r] = (VT)t;
  y[r] = (VT)((AT)y[r] + (AT)ck * t);
}

// degree 0: y = [y +] c0 w0
template <typename VT, typename RT>
__global__ void k_scale_add(int n, const RT* __restrict__ w0, VT* __restrict__ y, double c0, int accum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  VT v = (VT)c0 * (VT)w0[i];
  if (accum) v += y[i];
  y[i] = v;
}

// ------------------------------------------------------------------ residual, transfer
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(TPB) k_residual(Mat<MT> A, const RT* __restrict__ f, const VT* __restrict__ x,
                                                  VT* __restrict__ s) {
  using AT = VT;
  const int r = row_of(A);
  if (r < 0) return;
  const AT ax = (AT)A.D[r] * (AT)x[r] - offdiag<AT>(A, r, x);
  s[r] = (VT)((AT)f[r] - ax);
}

// FP64 residual with its squared norm: s = f - A x, scal[slot] = (s, s).
__global__ void __launch_bounds__(TPB) k_residual_dot(Mat<double> A, const double* __restrict__ f,
                                                      const double* __restrict__ x, double* __restrict__ s,
                                                      double* partials, unsigned* counter, double* scal, Slots out) {
  const int r = row_of(A);
  double v[1] = {0.0};
  if (r >= 0) {
    const double res = f[r] - (A.D[r] * x[r] - offdiag<double>(A, r, x));
    s[r] = res;
    v[0] = res * res;
  }
  grid_sum_finish<1>(v, partials, counter, scal, out);
}

template <typename VT>
__global__ void k_restrict(int nc, const int* __restrict__ members, const int* __restrict__ off,
                           const VT* __restrict__ s, VT* __restrict__ b) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  VT acc = 0;
  for (int k = off[I]; k < off[I + 1]; ++k) acc += s[members[k]];
  b[I] = acc;
}

template <typename VT>
__global__ void k_prolong(int n, const int* __restrict__ agg, const VT* __restrict__ e, VT* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += e[agg[i]];
}

// ------------------------------------------------------------------ coarsest solve
// L y = b, L^T x = y with the dense factor; one wavefront, lane i owns row i.
template <typename VT, typename RT>
__global__ void __launch_bounds__(64) k_chol_solve_wave(int n, const double* __restrict__ Lg, const RT* __restrict__ b,
                                                        VT* __restrict__ x) {
  __shared__ double Ls[64 * 65];
  const int lane = threadIdx.x;
  for (int t = lane; t < n * n; t += 64) Ls[(t / n) * 65 + (t % n)] = Lg[t];
  __syncthreads();
  double bi = lane < n ? (double)b[lane] : 0.0;
  for (int k = 0; k < n; ++k) {
    const double yk = __shfl(bi, k, 64) / Ls[k * 65 + k];
    if (lane == k) bi = yk;
    else if (lane > k && lane < n) bi -= Ls[lane * 65 + k] * yk;
  }
  for (int k = n - 1; k >= 0; --k) {
    const double xk = __shfl(bi, k, 64) / Ls[k * 65 + k];
    if (lane == k) bi = xk;
    else if (lane < k) bi -= Ls[k * 65 + lane] * xk;
  }
  if (lane < n) x[lane] = (VT)bi;
}

// Same for larger coarsest levels: one workgroup, the vector in LDS.
template <typename VT, typename RT>
__global__ void __launch_bounds__(TPB) k_chol_solve_block(int n, const double* __restrict__ Lg,
                                                          const RT* __restrict__ b, VT* __restrict__ x) {
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

// ------------------------------------------------------------------ flexible CG
// scal[dots.s[i]] = (z, q_i) for i < k.
template <typename ZT, typename QT>
__global__ void __launch_bounds__(TPB) k_multidot(int n, const ZT* __restrict__ z, VecPtrs qs, int k,
                                                  double* partials, unsigned* counter, double* scal, Slots dots) {
  double v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double zj = (double)z[j];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < k) v[i] += zj * (double)static_cast<const QT*>(qs.p[i])[j];
  }
  grid_sum_finish<8>(v, partials, counter, scal, dots);
}

// p = z - sum_i (dots_i / rho_i) p_i  (term dropped when rho_i <= 0); FP64 arithmetic.
template <typename PT, typename ZT>
__global__ void __launch_bounds__(TPB) k_fcg_p(int n, PT* p, const ZT* z, VecPtrs ps, int k, const double* scal,
                                               Slots dots, Slots rhos) {
  __shared__ double beta[8];
  if (threadIdx.x < 8) {
    const int i = threadIdx.x;
    double b = 0.0;
    if (i < k) {
      const double rho = scal[rhos.s[i]];
      b = rho > 0.0 ? scal[dots.s[i]] / rho : 0.0;
    }
    beta[i] = b;
  }
  __syncthreads();
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double v = (double)z[j];
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < k) v -= beta[i] * (double)static_cast<const PT*>(ps.p[i])[j];
    p[j] = (PT)v;
  }
}

// q = A p; scal[out.s[0]] = (p, q), scal[out.s[1]] = (p, r).
template <typename VT, typename MT, typename RT>
__global__ void __launch_bounds__(TPB) k_spmv_dots(Mat<MT> A, const VT* __restrict__ p, VT* __restrict__ q,
                                                   const RT* __restrict__ rv, double* partials, unsigned* counter,
                                                   double* scal, Slots out) {
  using AT = VT;
  const int r = row_of(A);
  double v[2] = {0.0, 0.0};
  if (r >= 0) {
    const AT pr = (AT)p[r];
    const AT ap = (AT)A.D[r] * pr - offdiag<AT>(A, r, p);
    q[r] = (VT)ap;
    v[0] = (double)pr * (double)ap;
    v[1] = (double)pr * (double)rv[r];
  }
  grid_sum_finish<2>(v, partials, counter, scal, out);
}

// alpha = gamma / rho (0 if rho <= 0 or not finite); x (= or +=) alpha p;
// optionally r -= alpha q and scal[s_rr] = (r, r).
template <typename VT, typename PT, bool RR>
__global__ void __launch_bounds__(TPB) k_fcg_xr(int n, const PT* __restrict__ p, const VT* __restrict__ q,
                                                VT* __restrict__ x, VT* __restrict__ r, const double* scal_in,
                                                int s_rho, int s_gam, int x_init, int upd_r, double* partials,
                                                unsigned* counter, double* scal, Slots rr_slot) {
  const double rho = scal_in[s_rho];
  const double alpha = (rho > 0.0 && isfinite(rho)) ? scal_in[s_gam] / rho : 0.0;
  double v[1] = {0.0};
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double pj = (double)p[j];
    x[j] = (VT)(x_init ? alpha * pj : (double)x[j] + alpha * pj);
    if (upd_r) {
      const double rj = (double)r[j] - alpha * (double)q[j];
      r[j] = (VT)rj;
      if (RR) v[0] += rj * rj;
    }
  }
  if (RR) grid_sum_finish<1>(v, partials, counter, scal, rr_slot);
}

template <typename A, typename B>
__global__ void k_convert(int n, const A* __restrict__ a, B* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (B)a[i];
}

__global__ void k_zero_u32(unsigned* c) { *c = 0u; }

// ------------------------------------------------------------------ host orchestration
Slots slots1(int a) { Slots s; for (int i = 0; i < 8; ++i) s.s[i] = S_DUMMY; s.s[0] = a; return s; }
Slots slots2(int a, int b) { Slots s = slots1(a); s.s[1] = b; return s; }
Slots slots_range(int base, int k) {
  Slots s;
  for (int i = 0; i < 8; ++i) s.s[i] = i < k ? base + i : S_DUMMY;
  return s;
}

template <typename VT, typename MT>
struct Engine {
  amg_hier* h;
  hipStream_t s;

  Mat<MT> A(int l) const { return mat_of<MT>(h->lv[l]); }
  VT* wsv(void* p) const { return static_cast<VT*>(p); }

  template <typename RT>
  int32_t smooth(int l, const RT* r, VT* y, bool accum) {
    const Level& lv = h->lv[l];
    const int m = h->p.degree;
    const auto Am = A(l);
    const double theta = lv.theta, inv_eta = 1.0 / lv.eta;
    const double* c = lv.coef.data();
    if (m == 0) {
      hipLaunchKernelGGL((k_scale_add<VT, RT>), dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, r, y, c[0], (int)accum);
      AMG_HIP(hipGetLastError());
      return AMG_OK;
    }
    VT* bufA = wsv(h->ws[l].A);
    VT* bufB = wsv(h->ws[l].B);
    hipLaunchKernelGGL((k_cheb_first<VT, MT, RT>), dim3(Am.nb), dim3(TPB), 0, s, Am, r, bufA, y, theta, inv_eta,
                       c[0], c[1], (int)accum, (int)(m > 1));
    VT* cur = bufA;
    VT* prevbuf = nullptr;  // buffer holding w_{k-1} for k >= 2
    for (int k = 1; k < m; ++k) {
      const int store = (k + 1 < m);
      VT* next;
      if (k == 1) {
        next = bufB;
        hipLaunchKernelGGL((k_cheb_next<VT, MT, RT>), dim3(Am.nb), dim3(TPB), 0, s, Am, cur, r, next, y, theta,
                           2.0 * inv_eta, c[k + 1], store);
      } else {
        next = prevbuf;
        hipLaunchKernelGGL((k_cheb_next<VT, MT, VT>), dim3(Am.nb), dim3(TPB), 0, s, Am, cur, prevbuf, next, y,
                           theta, 2.0 * inv_eta, c[k + 1], store);
      }
      prevbuf = cur;
      cur = next;
    }
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  template <typename RT>
  int32_t residual(int l, const RT* f, const VT* x, VT* out) {
    const auto Am = A(l);
    hipLaunchKernelGGL((k_residual<VT, MT, RT>), dim3(Am.nb), dim3(TPB), 0, s, Am, f, x, out);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  int32_t restrict_(int l, const VT* sv, VT* b) {
    const Level& lv = h->lv[l];
    const int nc = h->lv[l + 1].n;
    hipLaunchKernelGGL((k_restrict<VT>), dim3(nblk(nc)), dim3(TPB), 0, s, nc, lv.members, lv.member_off, sv, b);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  int32_t prolong(int l, const VT* e, VT* x) {
    const Level& lv = h->lv[l];
    hipLaunchKernelGGL((k_prolong<VT>), dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, lv.agg, e, x);
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  template <typename RT>
  int32_t coarse(const RT* b, VT* x) {
    const int n = h->nL;
    if (n <= 64) {
      hipLaunchKernelGGL((k_chol_solve_wave<VT, RT>), dim3(1), dim3(64), 0, s, n, h->chol, b, x);
    } else {
      hipLaunchKernelGGL((k_chol_solve_block<VT, RT>), dim3(1), dim3(TPB), sizeof(double) * n, s, n, h->chol, b, x);
    }
    AMG_HIP(hipGetLastError());
    return AMG_OK;
  }

  // z = Kcycle(l, r)
  template <typename RT>
  int32_t kcycle(int l, const RT* r, VT* x) {
    if (l == h->L) return coarse(r, x);
    VT* S = wsv(h->ws[l].S);
    VT* b = wsv(h->ws[l + 1].rhs);
    VT* e = wsv(h->ws[l + 1].sol);
    AMG_TRY(smooth(l, r, x, false));
    AMG_TRY(residual(l, r, x, S));
    AMG_TRY(restrict_(l, S, b));
    if (l + 1 == h->L) {
      AMG_TRY(coarse(static_cast<const VT*>(b), e));
    } else {
      AMG_TRY(inner(l + 1));
    }
    AMG_TRY(prolong(l, e, x));
    AMG_TRY(residual(l, r, x, S));
    AMG_TRY(smooth(l, static_cast<const VT*>(S), x, true));
    return AMG_OK;
  }

  // exactly nu flexible-CG steps from zero on level l (1 <= l < L): rhs -> sol
  int32_t inner(int l) {
    const int nu = h->p.inner_steps;
    const Level& lv = h->lv[l];
    const int n = lv.n;
    const auto Am = A(l);
    auto& W = h->ws[l];
    VT* rhs = wsv(W.rhs);
    VT* sol = wsv(W.sol);
    const int base = lbase(l);
    for (int k = 0; k < nu; ++k) {
      VT* z = wsv(W.Z[k]);
      AMG_TRY(kcycle(l, static_cast<const VT*>(rhs), z));
      if (k > 0) {
        VecPtrs qs{}, ps{};
        for (int i = 0; i < k; ++i) { qs.p[i] = W.Q[i]; ps.p[i] = W.Z[i]; }
        hipLaunchKernelGGL((k_multidot<VT, VT>), dim3(rblk(n)), dim3(TPB), 0, s, n, z, qs, k, h->partials,
                           h->counter, h->scal, slots_range(base + 16, k));
        hipLaunchKernelGGL((k_fcg_p<VT, VT>), dim3(rblk(n)), dim3(TPB), 0, s, n, z, z, ps, k, h->scal,
                           slots_range(base + 16, k), slots_range(base, k));
      }
      VT* q = wsv(W.Q[k]);
      hipLaunchKernelGGL((k_spmv_dots<VT, MT, VT>), dim3(Am.nb), dim3(TPB), 0, s, Am, z, q, rhs, h->partials,
                         h->counter, h->scal, slots2(base + k, base + 8 + k));
      hipLaunchKernelGGL((k_fcg_xr<VT, VT, false>), dim3(rblk(n)), dim3(TPB), 0, s, n, z, q, sol, rhs, h->scal,
                         base + k, base + 8 + k, (int)(k == 0), (int)(k + 1 < nu), h->partials, h->counter,
                         h->scal, slots1(S_DUMMY));
      AMG_HIP(hipGetLastError());
    }
    return AMG_OK;
  }

  // one outer iteration at window position j; u, r FP64 (finest level)
  int32_t outer_iter(int j, double* u) {
    const int n = h->lv[0].n;
    const auto A64 = mat_of<double>(h->lv[0]);
    VT* z = wsv(h->z);
    AMG_TRY(kcycle(0, static_cast<const double*>(h->r), z));
    VecPtrs qs{}, ps{};
    for (int i = 0; i < j; ++i) { qs.p[i] = h->Qo[i]; ps.p[i] = h->P[i]; }
    if (j > 0) {
      hipLaunchKernelGGL((k_multidot<VT, double>), dim3(rblk(n)), dim3(TPB), 0, s, n, z, qs, j, h->partials,
                         h->counter, h->scal, slots_range(S_DOTS, j));
    }
    hipLaunchKernelGGL((k_fcg_p<double, VT>), dim3(rblk(n)), dim3(TPB), 0, s, n, h->P[j], z, ps, j, h->scal,
                       slots_range(S_DOTS, j), slots_range(S_RHOW, j));
    hipLaunchKernelGGL((k_spmv_dots<double, double, double>), dim3(A64.nb), dim3(TPB), 0, s, A64, h->P[j], h->Qo[j],
                       h->r, h->partials, h->counter, h->scal, slots2(S_RHOW + j, S_GAM));
    hipLaunchKernelGGL((k_fcg_xr<double, double, true>), dim3(rblk(n)), dim3(TPB), 0, s, n, h->P[j], h->Qo[j], u,
                       h->r, h->scal, S_RHOW + j, S_GAM, 0, 1, h->partials, h->counter, h->scal, slots1(S_RR));
    AMG_HIP(hipGetLastError());
    // stopping test inputs: (r, r) and rho_j
    AMG_HIP(hipMemcpyAsync(h->host_scal, h->scal + S_RR, sizeof(double), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipMemcpyAsync(h->host_scal + 1, h->scal + S_RHOW + j, sizeof(double), hipMemcpyDeviceToHost, s));
    return AMG_OK;
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

template <typename VT, typename MT>
int32_t solve_impl(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info) {
  auto t0 = clk::now();
  const int n = h->lv[0].n;
  const auto A64 = mat_of<double>(h->lv[0]);
  Engine<VT, MT> E{h, s};
  // r = f - A u, rr0
  hipLaunchKernelGGL(k_residual_dot, dim3(A64.nb), dim3(TPB), 0, s, A64, f, u, h->r, h->partials, h->counter,
                     h->scal, slots1(S_RR0));
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipMemcpyAsync(h->host_scal, h->scal + S_RR0, sizeof(double), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  const double rho0 = std::sqrt(h->host_scal[0]);
  int32_t status = AMG_OK;
  int it = 0;
  double rel = rho0 > 0.0 ? 1.0 : 0.0;
  if (rho0 > 0.0) {
    const bool use_graph = h->p.use_graph != 0;
    if (use_graph && (!h->graphs_ready || h->graph_u != u)) {
      AMG_TRY(capture_graphs<VT, MT>(h, u));
      h->graph_u = u;
    }
    status = AMG_ERR_MAXIT;
    for (it = 1; it <= h->p.max_iter; ++it) {
      const int j = (it - 1) % h->p.restart;
      if (use_graph) {
        AMG_HIP(hipGraphLaunch(h->iter_exec[j], s));
      } else {
        AMG_TRY(E.outer_iter(j, u));
      }
      AMG_HIP(hipStreamSynchronize(s));
      const double rr = h->host_scal[0], rho = h->host_scal[1];
      if (!(rho > 0.0) || !std::isfinite(rho)) {
        status = AMG_ERR_BREAKDOWN;
        break;
      }
      rel = std::sqrt(rr) / rho0;
      if (rel <= h->p.tol) {
        status = AMG_OK;
        break;
      }
    }
    if (it > h->p.max_iter) it = h->p.max_iter;
  }
  // true FP64 residual of the returned u
  hipLaunchKernelGGL(k_residual_dot, dim3(A64.nb), dim3(TPB), 0, s, A64, f, u, h->tmp, h->partials, h->counter,
                     h->scal, slots1(S_RRT));
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipMemcpyAsync(h->host_scal + 2, h->scal + S_RRT, sizeof(double), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  if (info) {
    info->status = status;
    info->iters = it;
    info->rel_res = rel;
    info->rel_res_true = rho0 > 0.0 ? std::sqrt(h->host_scal[2]) / rho0 : 0.0;
    info->solve_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  }
  (void)n;
  return status;
}

}  // namespace

void destroy_graphs(amg_hier* h) {
  for (int j = 0; j < 8; ++j) {
    if (h->iter_exec[j]) (void)hipGraphExecDestroy(h->iter_exec[j]);
    h->iter_exec[j] = nullptr;
  }
  h->graphs_ready = false;
}

int32_t prepare_solve(amg_hier* h, hipStream_t s) {
  for (int l = 0; l < std::max(h->L, 1); ++l) {
    const Level& lv = h->lv[l];
    if (!lv.sell_off || !lv.sell_w || !lv.sell_col || !lv.sell_val || !lv.D || (h->mixed && (!lv.sell_valf || !lv.Df))) {
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
    }
  }
  const size_t n0 = h->lv[0].n;
  AMG_TRY(dalloc(h, &h->r, n0));
  AMG_TRY(dalloc(h, &h->tmp, n0));
  AMG_TRY(dalloc(h, &h->z, n0 * vt + 16));
  for (int j = 0; j < h->p.restart; ++j) {
    AMG_TRY(dalloc(h, &h->P[j], n0));
    AMG_TRY(dalloc(h, &h->Qo[j], n0));
  }
  h->max_blocks = std::max(RED_BLOCKS, nblk(n0));
  AMG_TRY(dalloc(h, &h->partials, (size_t)h->max_blocks * 8));
  AMG_TRY(dalloc(h, &h->scal, SCAL_SIZE));
  AMG_TRY(dalloc(h, &h->counter, 1));
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, h->counter);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipHostMalloc((void**)&h->host_scal, 64 * sizeof(double), hipHostMallocDefault));
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

int32_t solve(amg_hier* h, const double* f, double* u, hipStream_t s, amg_info* info) {
  if (h->mixed) return solve_impl<float, float>(h, f, u, s, info);
  return solve_impl<double, double>(h, f, u, s, info);
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
