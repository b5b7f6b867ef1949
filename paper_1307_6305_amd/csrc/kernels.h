// Device code shared by the single-solve and the batched executors: level
// views, the per-row steps of the cycle, the coarsest solve, and the
// interpreter of recorded op programs that runs a small level's inner solve
// out of one workgroup's LDS.
#pragma once

#include <algorithm>
#include <cstdint>

#include "device_util.h"
#include "hier.h"

namespace amg {

constexpr int TPB = 256;
constexpr int TAIL_THREADS = 1024;

// Scalar area.  Outer iteration: rr, (p,r), window dots, window rho.
// Inner solve on level l: base(l) + [0,8) rho_k, [8,16) gamma_k, [16,24) dots.
constexpr int S_RR = 0, S_XR = 1, S_GAM = 2, S_RR0 = 3, S_RRT = 4, S_FF = 5, S_DUMMY = 7, S_DOTS = 8, S_RHOW = 16;
inline int lbase(int l) { return 64 + 32 * l; }
constexpr int SCAL_SIZE = 64 + 32 * (AMG_MAX_LEVELS + 1);

inline int nblk(int64_t n, int tpb = TPB) { return (int)std::max<int64_t>(1, (n + tpb - 1) / tpb); }

struct VecPtrs {
  const void* p[8];
};

// A level's matrix in its sliced-ELL layout.  Row-parallel kernels cover the
// level in tiles of TPB rows, with (TPB << lk) threads per tile: K = 2^lk
// lanes per row.
template <typename MT>
struct Mat {
  int n;
  int nb;  // tiles of TPB rows
  int lc;  // log2 slice height
  int lk;  // log2 lanes per row
  const int* off;
  const int* width;
  const int* col;
  const MT* val;
  const MT* D;
  const int* perm;  // slot -> row inside each 64-row group, or null (identity)
};

struct Transfer {
  int n, nc;
  const int* agg;
  const int* members;
  const int* member_off;
};

struct CoarseView {
  int n;
  const double* Linv;   // inverse of the Cholesky factor, row-major (lower)
  const double* LinvT;  // its transpose
};

template <typename MT>
Mat<MT> mat_of(const Level& lv);
template <>
inline Mat<double> mat_of<double>(const Level& lv) {
  return Mat<double>{lv.n, nblk(lv.n), lv.sell_lc, lv.sell_lk, lv.sell_off, lv.sell_w, lv.sell_col, lv.sell_val,
                     lv.D, lv.sell_perm};
}
template <>
inline Mat<float> mat_of<float>(const Level& lv) {
  return Mat<float>{lv.n, nblk(lv.n), lv.sell_lc, lv.sell_lk, lv.sell_off, lv.sell_w, lv.sell_col, lv.sell_valf,
                    lv.Df, lv.sell_perm};
}

// The level's plain layout (the tail program's); null arrays if it has none.
template <typename MT>
Mat<MT> plain_mat_of(const Level& lv);
template <>
inline Mat<double> plain_mat_of<double>(const Level& lv) {
  return Mat<double>{lv.n, nblk(lv.n), 6, 0, lv.plain_off, lv.plain_w, lv.plain_col, lv.plain_val, lv.D, nullptr};
}
template <>
inline Mat<float> plain_mat_of<float>(const Level& lv) {
  return Mat<float>{lv.n, nblk(lv.n), 6, 0, lv.plain_off, lv.plain_w, lv.plain_col, lv.plain_valf, lv.Df, nullptr};
}

inline Transfer transfer_of(const amg_hier* h, int l) {
  const Level& lv = h->lv[l];
  return Transfer{lv.n, h->lv[l + 1].n, lv.agg, lv.members, lv.member_off};
}

// ------------------------------------------------------------------ per-row steps
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// A vector operand read at row j: the vector itself, or the vector plus the
// prolongation of a coarse correction, x_j + e_{agg(j)} (P piecewise
// constant), computed where it is read instead of in a pass of its own.
template <typename XT>
struct XPlain {
  const XT* __restrict__ x;
  __device__ __forceinline__ XT operator()(int j) const { return x[j]; }
};

template <typename VT>
struct XProlong {
  const VT* __restrict__ x;
  const VT* __restrict__ e;
  const int* __restrict__ agg;
  __device__ __forceinline__ VT operator()(int j) const { return x[j] + e[agg[j]]; }
};

// Flexible-CG vector updates read where they are used instead of in a pass
// of their own.  Each computes exactly what the update step stores (FP64
// fused multiply-add, rounded to the vector type), so folding changes no bit.
//   XAxpy:  r_j - alpha q_j        (right-hand side after a step)
//   XDir:   z_j - beta p_j         (new direction against one earlier one)
//   CUpd:   x_a + alpha p_a        (inner solution after its last step)
template <typename VT>
__device__ __forceinline__ VT fcg_axpy(double a, double x, double y) {
  return (VT)__builtin_fma(a, x, y);
}

template <typename VT>
struct XAxpy {
  const VT* __restrict__ r;
  const VT* __restrict__ q;
  double alpha;
  __device__ __forceinline__ VT operator()(int j) const { return fcg_axpy<VT>(-alpha, (double)q[j], (double)r[j]); }
};

template <typename VT>
struct XDir {
  const VT* __restrict__ z;
  const VT* __restrict__ p;
  double beta;
  __device__ __forceinline__ VT operator()(int j) const { return fcg_axpy<VT>(-beta, (double)p[j], (double)z[j]); }
};

template <typename VT>
struct CUpd {
  const VT* __restrict__ x;
  const VT* __restrict__ p;
  double alpha;
  __device__ __forceinline__ VT operator()(int a) const { return fcg_axpy<VT>(alpha, (double)p[a], (double)x[a]); }
};

// x_j + e_{agg(j)} with the coarse correction e given by an accessor.
template <typename VT, typename CE>
struct XProlongC {
  const VT* __restrict__ x;
  CE e;
  const int* __restrict__ agg;
  __device__ __forceinline__ VT operator()(int j) const { return x[j] + e(agg[j]); }
};

// sum_j W_rj x_j over the stored entries of the row in `slot`, computed by
// the K lanes j = 0..K-1 of the slot together (every lane gets the sum).
// Entry k of the row goes to class k mod 8; each class is summed in order
// of k with fused multiply-adds, and the eight class sums are combined by the
// fixed tree ((c0 + c4) + (c2 + c6)) + ((c1 + c5) + (c3 + c7)).  Lane j holds
// the classes j, j + K, ..., so every K, slice height and row order gives the
// same bits.  The loads of U steps are issued together: steps past the slice
// width re-read its last step (a cache hit) and are not added.
template <int K, typename AT, typename MT, typename XA>
__device__ __forceinline__ AT offdiag_k(const Mat<MT>& A, int slot, int j, const XA& x) {
  constexpr int U = 8 / K;
  const int s = slot >> A.lc, p = slot & ((1 << A.lc) - 1);
  const int stride = K << A.lc;
  const int base = A.off[s] + p * K + j;
  const int* __restrict__ c = A.col + base;
  const MT* __restrict__ v = A.val + base;
  const int wd = A.width[s];
  AT acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = (AT)0;
  for (int t = 0; t < wd; t += U) {
    int cv[U];
    MT vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tt = min(t + u, wd - 1) * stride;
      cv[u] = c[tt];
      vv[u] = v[tt];
    }
    AT xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = (AT)x(cv[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (t + u < wd) acc[u] = fmadd((AT)vv[u], (AT)xv[u], acc[u]);
  }
  AT sum;
  if constexpr (K == 1) {
    sum = ((acc[0] + acc[4]) + (acc[2] + acc[6])) + ((acc[1] + acc[5]) + (acc[3] + acc[7]));
  } else if constexpr (K == 2) {
    sum = (acc[0] + acc[2]) + (acc[1] + acc[3]);
    sum += __shfl_xor(sum, 1, 64);
  } else {
    sum = acc[0] + acc[1];
    sum += __shfl_xor(sum, 2, 64);
    sum += __shfl_xor(sum, 1, 64);
  }
  return sum;
}

// The off-diagonal sum of the row in `slot` on the level's layout (K lanes).
template <typename AT, typename MT, typename XA>
__device__ __forceinline__ AT offdiag_a(const Mat<MT>& A, int slot, int j, const XA& x) {
  if (A.lk == 0) return offdiag_k<1, AT>(A, slot, j, x);
  if (A.lk == 1) return offdiag_k<2, AT>(A, slot, j, x);
  return offdiag_k<4, AT>(A, slot, j, x);
}

template <typename AT, typename MT, typename XT>
__device__ __forceinline__ AT offdiag(const Mat<MT>& A, int slot, int j, const XT* __restrict__ x) {
  return offdiag_a<AT>(A, slot, j, XPlain<XT>{x});
}

// Where a row step takes its off-diagonal sum from: the matrix in its layout
// (OffMat), entries a caller has already loaded for this lane (OffPre: rows
// whose slice is at most one batch of 8 / K entries per lane wide, the loads
// offdiag_k issues for its first and only batch, added the same way -- the
// same bits), or the tail program's uniform-width layout in LDS (OffTail).
// The batched executor loads a row's entries once and applies them to every
// right-hand side that shares the matrix.
struct OffMat {
  template <typename AT, typename MT, typename XA>
  __device__ __forceinline__ AT sum(const Mat<MT>& A, int slot, int j, const XA& x) const {
    return offdiag_a<AT>(A, slot, j, x);
  }
};

template <int K, typename MT>
struct OffPre {
  static constexpr int U = 8 / K;
  int cv[U];
  MT vv[U];
  int wd;  // the slice's width in steps of the lane (<= U)
  // the entries of the lane of `slot` (its one batch), as offdiag_k loads them
  __device__ __forceinline__ void load(const Mat<MT>& A, int slot, int j) {
    const int s = slot >> A.lc, p = slot & ((1 << A.lc) - 1);
    const int stride = K << A.lc;
    const int base = A.off[s] + p * K + j;
    wd = A.width[s];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tt = min(u, wd - 1) * stride;
      cv[u] = A.col[base + tt];
      vv[u] = A.val[base + tt];
    }
  }
  template <typename AT, typename MT2, typename XA>
  __device__ __forceinline__ AT sum(const Mat<MT2>&, int, int, const XA& x) const {
    AT acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = (AT)0;
    AT xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = (AT)x(cv[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < wd) acc[u] = fmadd((AT)vv[u], (AT)xv[u], acc[u]);
    AT sum;
    if constexpr (K == 1) {
      sum = ((acc[0] + acc[4]) + (acc[2] + acc[6])) + ((acc[1] + acc[5]) + (acc[3] + acc[7]));
    } else if constexpr (K == 2) {
      sum = (acc[0] + acc[2]) + (acc[1] + acc[3]);
      sum += __shfl_xor(sum, 1, 64);
    } else {
      sum = acc[0] + acc[1];
      sum += __shfl_xor(sum, 2, 64);
      sum += __shfl_xor(sum, 1, 64);
    }
    return sum;
  }
};

// The tail program's matrices: 64-row slices of one width PW for the whole
// level (a multiple of 4; short rows padded with zero weights on the row's
// own column), entry t of row r at ((r >> 6) * PW + t) * 64 + (r & 63), so
// that no per-slice offset or width is read.  All loads of a row's entries
// are issued before any product is formed, and the products go to four
// chains, entry t to chain t mod 4, added at the end as (c0 + c1) + (c2 + c3)
// -- the tail's own fixed order, whichever code path below runs.
template <int PW, typename AT, typename MT, typename XA>
__device__ __forceinline__ AT rowsum_pw(const int* __restrict__ c, const MT* __restrict__ v, const XA& x) {
  int cc[PW];
  AT vv[PW], xx[PW];
#pragma unroll
  for (int t = 0; t < PW; ++t) cc[t] = c[t * 64];
#pragma unroll
  for (int t = 0; t < PW; ++t) vv[t] = (AT)v[t * 64];
#pragma unroll
  for (int t = 0; t < PW; ++t) xx[t] = (AT)x(cc[t]);
  AT a[4] = {(AT)0, (AT)0, (AT)0, (AT)0};
#pragma unroll
  for (int t = 0; t < PW; ++t) a[t & 3] = fmadd(vv[t], xx[t], a[t & 3]);
  return (a[0] + a[1]) + (a[2] + a[3]);
}

struct OffTail {
  int pw;
  template <typename AT, typename MT, typename XA>
  __device__ __forceinline__ AT sum(const Mat<MT>& A, int slot, int, const XA& x) const {
    const int base = (slot >> 6) * pw * 64 + (slot & 63);
    const int* __restrict__ c = A.col + base;
    const MT* __restrict__ v = A.val + base;
    switch (pw) {
      case 0:
        return (AT)0;
      case 4:
        return rowsum_pw<4, AT>(c, v, x);
      case 8:
        return rowsum_pw<8, AT>(c, v, x);
      case 12:
        return rowsum_pw<12, AT>(c, v, x);
      case 16:
        return rowsum_pw<16, AT>(c, v, x);
      default: {  // wider levels: four entries at a time, the same chains
        AT a[4] = {(AT)0, (AT)0, (AT)0, (AT)0};
        for (int t = 0; t < pw; t += 4) {
          int cc[4];
          AT vv[4], xx[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) cc[i] = c[(t + i) * 64];
#pragma unroll
          for (int i = 0; i < 4; ++i) vv[i] = (AT)v[(t + i) * 64];
#pragma unroll
          for (int i = 0; i < 4; ++i) xx[i] = (AT)x(cc[i]);
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = fmadd(vv[i], xx[i], a[i]);
        }
        return (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
  }
};

template <typename MT>
__device__ __forceinline__ int row_at(const Mat<MT>& A, int slot) {
  return A.perm ? A.perm[slot] : slot;
}

// The row steps below are called by all K lanes of a slot; lane 0 writes the
// row's results.
//
// w1 = (A w0 - theta w0) / eta;  y = [y +] c0 w0 + c1 w1   (c already divided by eta)
//
// With e and agg given (accumulating steps only), y holds x before the
// prolongation of a coarse correction: y is read as y_r + e_{agg(r)}.
template <typename VT, typename MT, typename RT, typename OD = OffMat>
__device__ __forceinline__ void row_cheb_first(const Mat<MT>& A, int slot, int j, const RT* __restrict__ w0, VT* w1,
                                               VT* y, double theta, double inv_eta, double c0, double c1, int accum,
                                               int store, const VT* __restrict__ e = nullptr,
                                               const int* __restrict__ agg = nullptr, const OD& od = OD()) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT x0 = (AT)w0[r];
  const AT d = (AT)A.D[r];
  const AT y0 = accum ? (AT)(e ? (VT)(y[r] + e[agg[r]]) : y[r]) : (AT)0;
  const AT off = od.template sum<AT>(A, slot, j, XPlain<RT>{w0});
  if (j) return;
  const AT ax = d * x0 - off;
  const AT t = (ax - (AT)theta * x0) * (AT)inv_eta;
  if (store) w1[r] = (VT)t;
  AT yy = (AT)c0 * x0 + (AT)c1 * t;
  if (accum) yy += y0;
  y[r] = (VT)yy;
}

// The same step with w0 and the accumulated start value of y given by
// accessors (W0(j): w0 at row j; Y0(r): the value y is accumulated onto).
// Returns the row in the writing lane (-1 in the others) and its w0 value.
template <typename VT, typename MT, typename W0, typename Y0>
__device__ __forceinline__ int row_cheb_first_a(const Mat<MT>& A, int slot, int j, const W0& w0, VT* w1, VT* y,
                                                const Y0& yin, double theta, double inv_eta, double c0, double c1,
                                                int accum, int store, VT* w0_out) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT x0 = (AT)w0(r);
  const AT d = (AT)A.D[r];
  const AT y0 = accum ? (AT)yin(r) : (AT)0;
  const AT off = offdiag_a<AT>(A, slot, j, w0);
  if (j) return -1;
  const AT ax = d * x0 - off;
  const AT t = (ax - (AT)theta * x0) * (AT)inv_eta;
  if (store) w1[r] = (VT)t;
  AT yy = (AT)c0 * x0 + (AT)c1 * t;
  if (accum) yy += y0;
  y[r] = (VT)yy;
  *w0_out = (VT)x0;
  return r;
}

template <typename VT>
struct YPlain {
  const VT* __restrict__ y;
  __device__ __forceinline__ VT operator()(int r) const { return y[r]; }
};

template <typename VT, typename CE>
struct YFold {
  const VT* __restrict__ y;
  CE e;
  const int* __restrict__ agg;
  __device__ __forceinline__ VT operator()(int r) const { return (VT)(y[r] + e(agg[r])); }
};

// Loads and stores of operands a row step touches once (NT: non-temporal,
// i.e. streamed past the caches instead of displacing what is reused).
template <bool NT, typename T>
__device__ __forceinline__ T ld_row(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_row(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// w_{k+1} = 2 (A w_k - theta w_k) / eta - w_{k-1};  y += c_{k+1} w_{k+1}.
// wnext may alias wprev (each element is read before it is overwritten).
// NT (levels far larger than the caches): the row's own operands D_r,
// w_{k-1,r}, y_r and its results are streamed non-temporally, so that the
// matrix and the gathered w_k stay cached; same arithmetic.
template <typename VT, typename MT, typename PT, bool NT = false, typename OD = OffMat>
__device__ __forceinline__ void row_cheb_next(const Mat<MT>& A, int slot, int j, const VT* __restrict__ wk,
                                              const PT* wprev, VT* wnext, VT* y, double theta, double two_inv_eta,
                                              double ck, int store, const OD& od = OD(), VT* y_out = nullptr) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT xk = (AT)wk[r];
  const AT d = (AT)ld_row<NT>(A.D + r);
  const AT wp = (AT)ld_row<NT>(wprev + r);
  const AT y0 = (AT)ld_row<NT>(y + r);
  const AT off = od.template sum<AT>(A, slot, j, XPlain<VT>{wk});
  if (j) return;
  const AT ax = d * xk - off;
  const AT t = (ax - (AT)theta * xk) * (AT)two_inv_eta - wp;
  if (store) st_row<NT>(wnext + r, (VT)t);
  const VT yv = (VT)(y0 + (AT)ck * t);
  st_row<NT>(y + r, yv);
  if (y_out) *y_out = yv;  // the stored value, for a caller that goes on with it
}

// s = f - A x; returns the row in the writing lane, -1 in the others
template <typename VT, typename MT, typename RT, typename OD = OffMat>
__device__ __forceinline__ int row_residual(const Mat<MT>& A, int slot, int j, const RT* __restrict__ f,
                                            const VT* __restrict__ x, VT* s, const OD& od = OD()) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT xr = (AT)x[r];
  const AT d = (AT)A.D[r];
  const AT fr = (AT)f[r];
  const AT off = od.template sum<AT>(A, slot, j, XPlain<VT>{x});
  if (j) return -1;
  const AT ax = d * xr - off;
  s[r] = (VT)(fr - ax);
  return r;
}

// s = f - A (x + P e): the residual after the prolongation of the coarse
// correction e, without writing x + P e (the next smoothing step adds e).
template <typename VT, typename MT, typename RT, typename OD = OffMat>
__device__ __forceinline__ int row_residual_p(const Mat<MT>& A, int slot, int j, const RT* __restrict__ f,
                                              const VT* __restrict__ x, const VT* __restrict__ e,
                                              const int* __restrict__ agg, VT* s, const OD& od = OD()) {
  using AT = VT;
  const XProlong<VT> X{x, e, agg};
  const int r = row_at(A, slot);
  const AT xr = (AT)X(r);
  const AT d = (AT)A.D[r];
  const AT fr = (AT)f[r];
  const AT off = od.template sum<AT>(A, slot, j, X);
  if (j) return -1;
  const AT ax = d * xr - off;
  s[r] = (VT)(fr - ax);
  return r;
}

// s = f - A X with the operand given by an accessor (X(j): x_j, e.g.
// x_j + e_{agg(j)}).
template <typename VT, typename MT, typename RT, typename XA>
__device__ __forceinline__ int row_residual_a(const Mat<MT>& A, int slot, int j, const RT* __restrict__ f,
                                              const XA& X, VT* s) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT xr = (AT)X(r);
  const AT d = (AT)A.D[r];
  const AT fr = (AT)f[r];
  const AT off = offdiag_a<AT>(A, slot, j, X);
  if (j) return -1;
  const AT ax = d * xr - off;
  s[r] = (VT)(fr - ax);
  return r;
}

// The value f_r - (A x)_r of the row in `slot` (every lane gets it; the
// same arithmetic as row_residual).
template <typename VT, typename MT, typename RT>
__device__ __forceinline__ VT row_residual_value(const Mat<MT>& A, int slot, int j, const RT* __restrict__ f,
                                                 const VT* __restrict__ x, int r) {
  using AT = VT;
  const AT xr = (AT)x[r];
  const AT d = (AT)A.D[r];
  const AT fr = (AT)f[r];
  const AT off = offdiag<AT>(A, slot, j, x);
  const AT ax = d * xr - off;
  return (VT)(fr - ax);
}

// b_I = sum of s over the members of aggregate I in member order; the
// members' indices and values are loaded eight at a time, then added in
// order (the same sums as one at a time, without a serial chain of loads).
template <typename VT>
__device__ __forceinline__ void row_restrict(const Transfer& T, int I, const VT* __restrict__ s, VT* b) {
  constexpr int B = 8;
  VT acc = 0;
  int k = T.member_off[I];
  const int k1 = T.member_off[I + 1];
  for (; k + B <= k1; k += B) {
    int m[B];
    VT v[B];
#pragma unroll
    for (int i = 0; i < B; ++i) m[i] = T.members[k + i];
#pragma unroll
    for (int i = 0; i < B; ++i) v[i] = s[m[i]];
#pragma unroll
    for (int i = 0; i < B; ++i) acc += v[i];
  }
  for (; k < k1; ++k) acc += s[T.members[k]];
  b[I] = acc;
}

template <typename VT>
__device__ __forceinline__ void row_prolong(const Transfer& T, int i, const VT* __restrict__ e, VT* x) {
  x[i] += e[T.agg[i]];
}

// q = A p for the row in `slot`; the writing lane returns the row and sets
// v = (p_r q_r, p_r rv_r) in FP64, the other lanes return -1.
template <typename VT, typename MT, typename RT, typename OD = OffMat>
__device__ __forceinline__ int row_spmv_dots(const Mat<MT>& A, int slot, int j, const VT* __restrict__ p, VT* q,
                                             const RT* __restrict__ rv, double (&v)[2], const OD& od = OD()) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT pr = (AT)p[r];
  const AT d = (AT)A.D[r];
  const double rr = (double)rv[r];
  const AT off = od.template sum<AT>(A, slot, j, XPlain<VT>{p});
  if (j) return -1;
  const AT ap = d * pr - off;
  q[r] = (VT)ap;
  v[0] = (double)pr * (double)ap;
  v[1] = (double)pr * rr;
  return r;
}

// q = A P with the operand given by an accessor; also returns P_r in pr.
template <typename VT, typename MT, typename RT, typename PA>
__device__ __forceinline__ int row_spmv_dots_a(const Mat<MT>& A, int slot, int j, const PA& P, VT* q,
                                               const RT* __restrict__ rv, double (&v)[2], VT* pr_out) {
  using AT = VT;
  const int r = row_at(A, slot);
  const AT pr = (AT)P(r);
  const AT d = (AT)A.D[r];
  const double rr = (double)rv[r];
  const AT off = offdiag_a<AT>(A, slot, j, P);
  if (j) return -1;
  const AT ap = d * pr - off;
  q[r] = (VT)ap;
  v[0] = (double)pr * (double)ap;
  v[1] = (double)pr * rr;
  *pr_out = (VT)pr;
  return r;
}

// Per-row values of one tile of ROWS rows, moved so that thread t < ROWS
// holds those of row tile * ROWS + t (zero elsewhere): a following block
// reduction then adds them in row order whatever the layout.  `rel` is the
// tile-relative row of the calling lane's values, or -1.  Call from every
// thread of the block.
template <int NV, int ROWS = TPB>
__device__ __forceinline__ void tile_stage(double (&v)[NV], int rel, double* stage) {
  for (int i = threadIdx.x; i < NV * ROWS; i += blockDim.x) stage[i] = 0.0;
  __syncthreads();
  if (rel >= 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) stage[k * ROWS + rel] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = threadIdx.x < ROWS ? stage[k * ROWS + threadIdx.x] : 0.0;
}

template <typename MT>
__device__ __forceinline__ bool needs_stage(const Mat<MT>& A) {
  return A.perm != nullptr || A.lk != 0;
}

__device__ __forceinline__ double fcg_alpha_of(double rho, double gam) {
  return (rho > 0.0 && isfinite(rho)) ? gam / rho : 0.0;
}
__device__ __forceinline__ double fcg_alpha(const double* scal, int s_rho, int s_gam) {
  return fcg_alpha_of(scal[s_rho], scal[s_gam]);
}

__device__ __forceinline__ double fcg_beta_of(double dot, double rho) { return rho > 0.0 ? dot / rho : 0.0; }
__device__ __forceinline__ double fcg_beta(const double* scal, int s_dot, int s_rho) {
  return fcg_beta_of(scal[s_dot], scal[s_rho]);
}

// Coarsest solve x = L^-T (L^-1 b) with the inverted factor: two triangular
// products.  For n <= 256 every product row is split into G = 4 partial sums
// (column classes j mod 4, each added in order over the full range of j --
// the factor's other triangle holds exact zeros, so the sums are unchanged),
// which are then added as (p0 + p1) + (p2 + p3): four times shorter chains.
// Larger n use one sum per row over its triangle.  The association depends
// only on n, not on the block size.  sb and sy hold 1024 doubles each.
// sum over j = j0, j0 + G, ... < n of M[j n + i] v[j], in that order, with
// eight products' loads in flight at a time
template <int G>
__device__ __forceinline__ double column_dot(const double* __restrict__ M, const double* v, int n, int i, int j0) {
  double acc = 0.0;
  int j = j0;
  for (; j + 7 * G < n; j += 8 * G) {
    double m[8], w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      m[q] = M[(size_t)(j + q * G) * n + i];
      w[q] = v[j + q * G];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += m[q] * w[q];
  }
  for (; j < n; j += G) acc += M[(size_t)j * n + i] * v[j];
  return acc;
}

template <typename VT, typename RT>
__device__ __forceinline__ void coarse_apply(const CoarseView& C, const RT* __restrict__ b, VT* x, double* sb,
                                             double* sy) {
  const int n = C.n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = (double)b[i];
  __syncthreads();
  if (n <= 256) {
    constexpr int G = 4;
    // y = L^-1 b: partials into sy, then y into sb
    for (int t = threadIdx.x; t < G * n; t += blockDim.x) {
      const int i = t / G, g = t % G;
      sy[t] = column_dot<G>(C.LinvT, sb, n, i, g);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      sb[i] = (sy[G * i] + sy[G * i + 1]) + (sy[G * i + 2] + sy[G * i + 3]);
    __syncthreads();
    // x = L^-T y
    for (int t = threadIdx.x; t < G * n; t += blockDim.x) {
      const int i = t / G, g = t % G;
      sy[t] = column_dot<G>(C.Linv, sb, n, i, g);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      x[i] = (VT)((sy[G * i] + sy[G * i + 1]) + (sy[G * i + 2] + sy[G * i + 3]));
    return;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = 0.0;
#pragma unroll 8
    for (int j = 0; j <= i; ++j) acc += C.LinvT[(size_t)j * n + i] * sb[j];
    sy[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = 0.0;
#pragma unroll 8
    for (int j = i; j < n; ++j) acc += C.Linv[(size_t)j * n + i] * sy[j];
    x[i] = (VT)acc;
  }
}

// ------------------------------------------------------------------ tail interpreter
enum OpType : int {
  OP_CHEB_FIRST = 1,
  OP_CHEB_NEXT,
  OP_SCALE_ADD,
  OP_RESIDUAL,
  OP_RESTRICT,
  OP_PROLONG,
  OP_COARSE,
  OP_MULTIDOT,
  OP_FCG_P,
  OP_SPMV_DOTS,
  OP_FCG_XR,
  OP_RESIDUAL_P,
};

// One op as the solver records it (host side, device addresses).
struct TailOp {
  int type, level, n, k;
  int i0, i1, i2, i3;
  double f0, f1, f2, f3;
  const void* a;
  const void* b;
  void* c;
  void* d;
  VecPtrs w;
  Slots s0, s1;
};

// One op as the tail interpreter reads it: every operand is a byte offset
// into the workgroup's LDS image, with the op's matrix and transfer map
// resolved when the program is laid out; an op on a level's matrix has the
// matrix's col, val and D offsets and, in `width`, its padded width PW (the
// uniform-width layout of OffTail; `off` is unused).  Fields by op:
//   CHEB_FIRST  a w0, c w1, d y, f0 theta, f1 1/eta, f2 c0, f3 c1, i0 accum,
//               i1 store, i2 fold (e = coarse correction, agg)
//   CHEB_NEXT   a w_k, b w_k-1, c w_k+1, d y, f0 theta, f1 2/eta, f2 c, i0 store
//   SCALE_ADD   a w0, d y, f0 c0, i0 accum
//   RESIDUAL    a f, b x, c s;  RESIDUAL_P the same with e, agg
//   RESTRICT    a s, c b, n coarse rows (members, member_off)
//   PROLONG     a e, c x (agg)
//   COARSE      a b, c x
//   MULTIDOT    a z, k; aux: k vector offsets, k destination slots (k = 1:
//               also b the vector, i0 the slot)
//   SPMV_DOTS   a p, b r, c q, i0 i1 destination slots
//   FCG_P       a z, c p, k; aux: k vector offsets, k dot slots, k rho slots
//               (k = 1: also b the vector, i0 the dot slot, i1 the rho slot)
//   FCG_XR      a p, b q, c x, d r, i0 rho slot, i1 gamma slot, i2 x_init, i3 update r
struct TailInstr {
  int type, n, k, i0;
  int i1, i2, i3;
  uint32_t aux;
  uint32_t a, b, c, d;
  uint32_t off, width, col, val;
  uint32_t D, agg, members, member_off;
  uint32_t e, pad0, pad1, pad2;
  double f0, f1, f2, f3;
};
static_assert(sizeof(TailInstr) == 128, "tail instructions are 128 bytes");

// Instructions stay in device memory, in this form (nothing to decode), and
// each op reads its own with scalar loads (constant address space: uniform,
// read-only) into scalar registers: neither LDS bandwidth nor vector
// registers, and every wave's per-op work on the scalar unit -- which the
// compute unit's waves share -- is a handful of instructions.  The kernel
// touches every line of the list once at start, so those reads hit the
// scalar cache.
typedef __attribute__((address_space(4))) const TailInstr ConstInstr;
typedef __attribute__((address_space(4))) const uint32_t ConstWord;

__device__ __forceinline__ TailInstr instr_load(const ConstInstr* p) {
  TailInstr I;
  ConstWord* w = reinterpret_cast<ConstWord*>(p);
  uint32_t* d = reinterpret_cast<uint32_t*>(&I);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(TailInstr) / 4); ++i) d[i] = w[i];
  return I;
}

struct TailCopy {
  const void* src;  // device address
  uint32_t dst;     // LDS byte offset
  int bytes;        // multiple of 16
};

// The tail program runs entirely out of the workgroup's LDS: its instruction
// list, the matrices, transfer maps, coarsest factor, vectors and scalars are
// laid out in one LDS image that the kernel fills from device memory at start;
// the tail level's solution is copied back at the end.
struct TailProgram {
  int nops;
  int ncin;
  const TailInstr* ops;  // instruction list (device memory)
  uint32_t scal_off;     // LDS offset of the scalar area
  const TailCopy* cin;
  TailCopy cout;  // solution of the tail level, LDS -> device
  uint32_t linv_off, linvt_off;  // inverse factor and its transpose (LDS)
  int nL;                        // coarsest size
  // When the program's last step (sol += alpha p) is folded into the copy-out:
  // LDS offset of p (0: plain copy), the step's scalar slots, row count.
  uint32_t fin_p;
  int fin_rho, fin_gam, fin_n;
};

template <typename T>
__device__ __forceinline__ T* lds_at(char* lds, uint32_t off) {
  return reinterpret_cast<T*>(lds + off);
}

template <typename MT>
__device__ __forceinline__ Mat<MT> instr_mat(const TailInstr& I, char* lds) {
  return Mat<MT>{I.n, 0, 6, 0, nullptr, nullptr, lds_at<const int>(lds, I.col), lds_at<const MT>(lds, I.val),
                 lds_at<const MT>(lds, I.D), nullptr};
}

// Runs a recorded program in one workgroup; every op is a data-parallel loop
// over rows followed by a workgroup barrier.  Reductions are workgroup
// reductions (no grid synchronization needed).
template <typename VT, typename MT>
__device__ __forceinline__ void run_tail(const TailProgram& P, char* lds, double* red, double* sb, double* sy,
                                         bool copy_constants) {
  const int tid = threadIdx.x, bd = blockDim.x;
  {
    // one scalar load per 64-byte line of the instruction list, the lines
    // dealt out over the wavefronts (the scalar cache is shared) so that each
    // has few loads in flight, overlapping the copy-in below; the value
    // itself is not needed
    ConstWord* w = (ConstWord*)(P.ops);
    const int lines = P.nops * (int)(sizeof(TailInstr) / 64);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), nwave = bd >> 6;
    uint32_t acc = 0;
#pragma unroll 16
    for (int l = wave; l < lines; l += nwave) acc ^= w[16 * l];
    __asm__ volatile("" : : "s"(acc));
  }
  for (int c = copy_constants ? 0 : P.ncin - 1; c < P.ncin; ++c) {
    const TailCopy cp = P.cin[c];
    const int4* __restrict__ src = static_cast<const int4*>(cp.src);
    int4* dst = reinterpret_cast<int4*>(lds + cp.dst);
    const int n16 = cp.bytes >> 4;
    int i = tid;
    for (; i + 3 * bd < n16; i += 4 * bd) {  // four loads in flight per thread
      const int4 a = src[i], b = src[i + bd], c2 = src[i + 2 * bd], d = src[i + 3 * bd];
      dst[i] = a;
      dst[i + bd] = b;
      dst[i + 2 * bd] = c2;
      dst[i + 3 * bd] = d;
    }
    for (; i < n16; i += bd) dst[i] = src[i];
  }
  __syncthreads();
  double* scal = lds_at<double>(lds, P.scal_off);
  const CoarseView C{P.nL, lds_at<const double>(lds, P.linv_off), lds_at<const double>(lds, P.linvt_off)};
  const ConstInstr* ops = (const ConstInstr*)(P.ops);
  for (int o = 0; o < P.nops; ++o) {
    const TailInstr I = instr_load(ops + o);
    switch (I.type) {
      case OP_CHEB_FIRST: {
        const Mat<MT> A = instr_mat<MT>(I, lds);
        const VT* w0 = lds_at<const VT>(lds, I.a);
        VT* w1 = lds_at<VT>(lds, I.c);
        VT* y = lds_at<VT>(lds, I.d);
        const VT* e = I.i2 ? lds_at<const VT>(lds, I.e) : nullptr;
        const int* agg = I.i2 ? lds_at<const int>(lds, I.agg) : nullptr;
        for (int r = tid; r < A.n; r += bd)
          row_cheb_first<VT, MT, VT, OffTail>(A, r, 0, w0, w1, y, I.f0, I.f1, I.f2, I.f3, I.i0, I.i1, e, agg,
                                                     OffTail{(int)I.width});
        break;
      }
      case OP_CHEB_NEXT: {
        const Mat<MT> A = instr_mat<MT>(I, lds);
        const VT* wk = lds_at<const VT>(lds, I.a);
        const VT* wp = lds_at<const VT>(lds, I.b);
        VT* wn = lds_at<VT>(lds, I.c);
        VT* y = lds_at<VT>(lds, I.d);
        for (int r = tid; r < A.n; r += bd)
          row_cheb_next<VT, MT, VT, false, OffTail>(A, r, 0, wk, wp, wn, y, I.f0, I.f1, I.f2, I.i0,
                                                           OffTail{(int)I.width});
        break;
      }
      case OP_SCALE_ADD: {
        const VT* w0 = lds_at<const VT>(lds, I.a);
        VT* y = lds_at<VT>(lds, I.d);
        for (int i = tid; i < I.n; i += bd) {
          VT v = (VT)I.f0 * w0[i];
          if (I.i0) v += y[i];
          y[i] = v;
        }
        break;
      }
      case OP_RESIDUAL: {
        const Mat<MT> A = instr_mat<MT>(I, lds);
        const VT* f = lds_at<const VT>(lds, I.a);
        const VT* x = lds_at<const VT>(lds, I.b);
        VT* sv = lds_at<VT>(lds, I.c);
        for (int r = tid; r < A.n; r += bd)
          (void)row_residual<VT, MT, VT, OffTail>(A, r, 0, f, x, sv, OffTail{(int)I.width});
        break;
      }
      case OP_RESIDUAL_P: {
        const Mat<MT> A = instr_mat<MT>(I, lds);
        const VT* f = lds_at<const VT>(lds, I.a);
        const VT* x = lds_at<const VT>(lds, I.b);
        const VT* e = lds_at<const VT>(lds, I.e);
        const int* agg = lds_at<const int>(lds, I.agg);
        VT* sv = lds_at<VT>(lds, I.c);
        for (int r = tid; r < A.n; r += bd)
          (void)row_residual_p<VT, MT, VT, OffTail>(A, r, 0, f, x, e, agg, sv, OffTail{(int)I.width});
        break;
      }
      case OP_RESTRICT: {
        const int* members = lds_at<const int>(lds, I.members);
        const int* moff = lds_at<const int>(lds, I.member_off);
        const VT* sv = lds_at<const VT>(lds, I.a);
        VT* b = lds_at<VT>(lds, I.c);
        for (int J = tid; J < I.n; J += bd) {
          VT acc = 0;
          int k = moff[J];
          const int k1 = moff[J + 1];
          if (k1 - k <= 16) {
            // every member's loads at once (indices clamped to the list),
            // added in member order: the same sums as one at a time
            const int last = k1 - 1;
            int m[16];
            VT v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) m[q] = members[min(k + q, last)];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = sv[m[q]];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc = k + q < k1 ? acc + v[q] : acc;
          } else {
            for (; k + 8 <= k1; k += 8) {  // eight members' loads in flight, added in order
              VT v[8];
#pragma unroll
              for (int q = 0; q < 8; ++q) v[q] = sv[members[k + q]];
#pragma unroll
              for (int q = 0; q < 8; ++q) acc += v[q];
            }
            for (; k < k1; ++k) acc += sv[members[k]];
          }
          b[J] = acc;
        }
        break;
      }
      case OP_PROLONG: {
        const int* agg = lds_at<const int>(lds, I.agg);
        const VT* e = lds_at<const VT>(lds, I.a);
        VT* x = lds_at<VT>(lds, I.c);
        for (int i = tid; i < I.n; i += bd) x[i] += e[agg[i]];
        break;
      }
      case OP_COARSE:
        coarse_apply<VT, VT>(C, lds_at<const VT>(lds, I.a), lds_at<VT>(lds, I.c), sb, sy);
        break;
      case OP_MULTIDOT: {
        if (I.k == 1) {  // one product: its operand and slot are in the instruction (b, i0)
          const VT* z = lds_at<const VT>(lds, I.a);
          const VT* q = lds_at<const VT>(lds, I.b);
          double v[1] = {0.0};
          for (int j = tid; j < I.n; j += bd) v[0] += (double)z[j] * (double)q[j];
          block_sum<1>(v, red);
          if (tid == 0) scal[I.i0] = v[0];
          break;
        }
        const uint32_t* vo = lds_at<const uint32_t>(lds, I.aux);
        const int* so = lds_at<const int>(lds, I.aux + 4 * I.k);
        uint32_t qo[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) qo[i] = i < I.k ? (uint32_t)__builtin_amdgcn_readfirstlane((int)vo[i]) : 0u;
        double v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.0;
        const VT* z = lds_at<const VT>(lds, I.a);
        for (int j = tid; j < I.n; j += bd) {
          const double zj = (double)z[j];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < I.k) v[i] += zj * (double)lds_at<const VT>(lds, qo[i])[j];
        }
        block_sum_k<8>(v, I.k, red);
        if (tid == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < I.k) scal[so[i]] = v[i];
        }
        break;
      }
      case OP_FCG_P: {
        if (I.k == 1) {  // one earlier direction: operand and slots in the instruction (b, i0, i1)
          const double beta = fcg_beta(scal, I.i0, I.i1);
          const VT* z = lds_at<const VT>(lds, I.a);
          const VT* po = lds_at<const VT>(lds, I.b);
          VT* p = lds_at<VT>(lds, I.c);
          for (int j = tid; j < I.n; j += bd) {
            double v = (double)z[j];
            v -= beta * (double)po[j];
            p[j] = (VT)v;
          }
          break;
        }
        const uint32_t* vo = lds_at<const uint32_t>(lds, I.aux);
        const int* sd = lds_at<const int>(lds, I.aux + 4 * I.k);
        const int* sr = lds_at<const int>(lds, I.aux + 8 * I.k);
        double beta[8];
        uint32_t po[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          beta[i] = i < I.k ? fcg_beta(scal, sd[i], sr[i]) : 0.0;
          po[i] = i < I.k ? (uint32_t)__builtin_amdgcn_readfirstlane((int)vo[i]) : 0u;
        }
        const VT* z = lds_at<const VT>(lds, I.a);
        VT* p = lds_at<VT>(lds, I.c);
        for (int j = tid; j < I.n; j += bd) {
          double v = (double)z[j];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < I.k) v -= beta[i] * (double)lds_at<const VT>(lds, po[i])[j];
          p[j] = (VT)v;
        }
        break;
      }
      case OP_SPMV_DOTS: {
        const Mat<MT> A = instr_mat<MT>(I, lds);
        const VT* p = lds_at<const VT>(lds, I.a);
        const VT* rv = lds_at<const VT>(lds, I.b);
        VT* q = lds_at<VT>(lds, I.c);
        double v[2] = {0.0, 0.0};
        for (int r = tid; r < A.n; r += bd) {
          double w[2];
          (void)row_spmv_dots<VT, MT, VT, OffTail>(A, r, 0, p, q, rv, w, OffTail{(int)I.width});
          v[0] += w[0];
          v[1] += w[1];
        }
        block_sum<2>(v, red);
        if (tid == 0) {
          scal[I.i0] = v[0];
          scal[I.i1] = v[1];
        }
        break;
      }
      case OP_FCG_XR: {
        const double alpha = fcg_alpha(scal, I.i0, I.i1);
        const VT* p = lds_at<const VT>(lds, I.a);
        const VT* q = lds_at<const VT>(lds, I.b);
        VT* x = lds_at<VT>(lds, I.c);
        VT* r = lds_at<VT>(lds, I.d);
        for (int j = tid; j < I.n; j += bd) {
          const double pj = (double)p[j];
          x[j] = (VT)(I.i2 ? alpha * pj : (double)x[j] + alpha * pj);
          if (I.i3) r[j] = (VT)((double)r[j] - alpha * (double)q[j]);
        }
        break;
      }
      default:
        break;
    }
    __syncthreads();
  }
  if (P.fin_p) {
    const double alpha = fcg_alpha(scal, P.fin_rho, P.fin_gam);
    const VT* x = lds_at<const VT>(lds, P.cout.dst);
    const VT* p = lds_at<const VT>(lds, P.fin_p);
    VT* dst = static_cast<VT*>(const_cast<void*>(P.cout.src));
    for (int i = tid; i < P.fin_n; i += bd) dst[i] = fcg_axpy<VT>(alpha, (double)p[i], (double)x[i]);
  } else {
    const int4* src = reinterpret_cast<const int4*>(lds + P.cout.dst);
    int4* dst = static_cast<int4*>(const_cast<void*>(P.cout.src));
    for (int i = tid; i < (P.cout.bytes >> 4); i += bd) dst[i] = src[i];
  }
}


}  // namespace amg
