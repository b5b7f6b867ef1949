// Device helpers: wavefront (64-lane) reductions and scans, deterministic
// block reductions, and the XCD-aware block remap.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg {

// splitmix64 (Steele, Lea and Flood): one output of the generator whose state
// is x.  The method's counter-based draws (independent-set priorities, power
// iteration start vectors) all come from it.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Sum over the 64 lanes of a wavefront; the result is valid in every lane.
// The shuffle tree is fixed, so the result is deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// A double moved across lanes by a DPP pattern (both 32-bit halves); lanes
// of rows outside ROWS get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The double sum over the 64 lanes through DPP lane moves (no LDS traffic):
// quad butterflies, the mirrors within 8 and 16 lanes, then the row
// broadcasts into rows 1, 3 and 2, 3; lane 63 ends with
// (R3 + R2) + (R1 + R0) of the row sums, which every lane returns.  The tree
// is fixed, so the result is deterministic.
template <>
__device__ __forceinline__ double wave_sum<double>(double v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

// red[0*K + k] + red[1*K + k] + ... + red[(nw-1)*K + k], added in that
// order: all sixteen slots are loaded at once (one LDS round trip instead of
// nw dependent ones), and the adds stop at nw (nw is uniform: a scalar
// branch per slot, no chain of selects through the unused ones).
template <int K>
__device__ __forceinline__ double wave_partials_sum(const double* red, int k, int nw) {
  double r[16];
#pragma unroll
  for (int w = 0; w < 16; ++w) r[w] = red[w * K + k];
  double s = r[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) {
    if (w >= nw) break;
    s += r[w];
  }
  return s;
}

// Block-wide sum of K values per thread (blockDim.x a multiple of 64, at most
// 1024).  Returns the totals in thread 0; `red` is LDS scratch of 16*K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[wid * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_partials_sum<K>(red, k, nw);
  }
}

// block_sum for the first kn of K values (the others are left as they are):
// the same tree, without the wavefront reductions of unused values.
template <int K>
__device__ __forceinline__ void block_sum_k(double (&v)[K], int kn, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k < kn) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kn) red[wid * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kn) v[k] = wave_partials_sum<K>(red, k, nw);
  }
}

// Up to 8 destination slots of a reduction in the hierarchy's scalar area.
struct Slots {
  int s[8];
};

// Where a grid reduction deposits its result.  Every block writes its partial
// sums to partials[block * K + k].  With `last_block` set, the last block to
// arrive (release/acquire ordering through `counter`) adds all partials and
// writes scal[slots.s[k]]; otherwise a separate one-block kernel
// (k_finish_sum) does it.  Large grids use the separate kernel: a fence per
// block costs an L2 write-back per block on this GPU.  Both paths add the
// partials in the same fixed order, so the result does not depend on which
// block arrives last nor on the path taken.
struct Red {
  double* partials;
  unsigned* counter;
  double* scal;
  Slots slots;
  int last_block;
};

constexpr int kFinishThreads = 256;

// Sum of partials[b*K + k] over b < nparts in a fixed order, by one block of
// kFinishThreads threads: thread t adds b = t, t + 256, ...; then the block tree.
// kn: only the first kn of the K values are summed (the rest are left 0).
template <int K>
__device__ __forceinline__ void sum_partials(const double* partials, int nparts, double (&acc)[K], double* red,
                                             int kn = K) {
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  if (threadIdx.x < kFinishThreads) {
    // B partials' loads in flight at once, then added in the same order as
    // one at a time (b, b + kFinishThreads, ...): the same sums
    constexpr int B = K <= 2 ? 8 : 4;
    int b = threadIdx.x;
    for (; b + (B - 1) * kFinishThreads < nparts; b += B * kFinishThreads) {
      double t[B][K];
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k) t[i][k] = k < kn ? partials[(b + i * kFinishThreads) * K + k] : 0.0;
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (k < kn) acc[k] += t[i][k];
    }
    for (; b < nparts; b += kFinishThreads) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kn) acc[k] += partials[b * K + k];
    }
  }
  block_sum_k<K>(acc, kn, red);
}

// Sums a producer left as per-block partials (a grid too large to finish in
// the kernel), finished at the start of the kernel that consumes them instead
// of in a launch of their own: every block forms the sums k_finish_sum would
// (sum_partials, the same order), block 0 also stores them into scal for later
// kernels, and every thread gets them in vals.  nparts = 0: nothing pending.
struct PendingSum {
  const double* partials;
  int nparts;
  int kn;
  Slots slots;
};

template <int K>
__device__ __forceinline__ void finish_pending(const PendingSum& ps, double* scal, double (&vals)[K]) {
  __shared__ double red[16 * 8];
  __shared__ double out[K];
  double acc[K];
  sum_partials<K>(ps.partials, ps.nparts, acc, red, ps.kn);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      out[k] = acc[k];
      if (blockIdx.x == 0 && k < ps.kn) scal[ps.slots.s[k]] = acc[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) vals[k] = out[k];
}

// kn: only the first kn values are summed (the rest are written as given).
// part: the block's partial slot (default: its block index; every slot of
// 0..gridDim.x-1 must be written by exactly one block).
template <int K>
__device__ __forceinline__ void grid_sum_finish(double (&v)[K], const Red& r, int kn = K, int part = -1) {
  __shared__ double red[16 * 8];
  __shared__ bool last;
  block_sum_k<K>(v, kn, red);
  if (threadIdx.x == 0) {
    const int b = part >= 0 ? part : (int)blockIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) r.partials[b * K + k] = v[k];
  }
  if (!r.last_block) return;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned t = atomicAdd(r.counter, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double acc[K];
  __syncthreads();
  sum_partials<K>(r.partials, gridDim.x, acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) r.scal[r.slots.s[k]] = acc[k];
    *r.counter = 0u;
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X.  This
// maps the hardware block id to a logical tile id such that every XCD works
// on one contiguous range of tiles (better reuse of its private L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int q = nblocks >> 3, r = nblocks & 7;
  const int x = bid & 7, k = bid >> 3;
  const int start = x * q + (x < r ? x : r);
  return start + k;
}

}  // namespace amg
