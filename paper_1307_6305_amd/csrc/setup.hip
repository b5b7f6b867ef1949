// Hierarchy construction on the device.
//
// Per level (Sections 2-4 of the paper): P matching passes, each on the
// quotient graph of the previous pass; the Galerkin operator of every pass as a
// per-coarse-row sort and reduce of the (agg_i, agg_j) pairs of the fine
// entries; the composite aggregate map and its member lists (restriction =
// segmented sum, prolongation = gather, P never stored); lambda1 = ||A||_inf;
// and finally the dense Cholesky factor of the coarsest matrix.
//
// Bit-exactness contract (matching and coarse operators): every quantity that
// decides the matching -- D_i, the edge strengths, the coarse weights -- is
// computed with correctly rounded binary64 operations in a fixed order (row
// sums left to right from d_i; strength (w*w)/(D_i*D_j) taken from the entry
// of row min(i, j); coarse sums in increasing fine row, then entry order).
// This file is compiled with -ffp-contract=off so that no multiply-add is
// fused.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>

#include "device_util.h"
#include "hier.h"

namespace amg {
namespace {

constexpr int TPB = 256;
inline int nblk(int64_t n, int tpb = TPB) { return (int)std::max<int64_t>(1, (n + tpb - 1) / tpb); }

// ------------------------------------------------------------------ temporaries
// Setup temporaries come from an arena: a few large device chunks carved
// into 256-byte aligned pieces, all returned when the arena goes out of
// scope (hipFree synchronizes the device; one per chunk instead of one per
// temporary).  release() gives a piece back when it and everything after it
// in its chunk have been released.
struct Temps {
  struct Piece {
    size_t off, bytes;
    bool freed;
  };
  struct Chunk {
    char* base;
    size_t size, used;
    std::vector<Piece> pieces;
  };
  std::vector<Chunk> chunks;
  static constexpr size_t kMinChunk = size_t(64) << 20;
  ~Temps() {
    for (auto& c : chunks) (void)hipFree(c.base);
  }
  template <typename T>
  int32_t get(T** p, size_t count) {
    const size_t bytes = (count * sizeof(T) + 16 + 255) & ~size_t(255);
    Chunk* c = chunks.empty() ? nullptr : &chunks.back();
    if (!c || c->used + bytes > c->size) {
      const size_t want = std::max(bytes, chunks.empty() ? kMinChunk : 2 * chunks.back().size);
      void* q = nullptr;
      hipError_t e = hipMalloc(&q, want);
      if (e != hipSuccess) {
        set_last_error(std::string("hipMalloc (setup temporary): ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;
      }
      chunks.push_back(Chunk{static_cast<char*>(q), want, 0, {}});
      c = &chunks.back();
    }
    c->pieces.push_back(Piece{c->used, bytes, false});
    *p = reinterpret_cast<T*>(c->base + c->used);
    c->used += bytes;
    return AMG_OK;
  }
  void release(void* p) {
    if (!p) return;
    for (auto& c : chunks) {
      char* q = static_cast<char*>(p);
      if (q < c.base || q >= c.base + c.size) continue;
      const size_t off = (size_t)(q - c.base);
      for (auto& pc : c.pieces)
        if (pc.off == off) pc.freed = true;
      while (!c.pieces.empty() && c.pieces.back().freed) {
        c.used = c.pieces.back().off;
        c.pieces.pop_back();
      }
      return;
    }
  }
};

// ------------------------------------------------------------------ generic kernels
__global__ void k_iota(int n, int* a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = i;
}

template <typename T>
__global__ void k_fill(size_t n, T* a, T v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// out_i = start_i + W[rp_i] + W[rp_i + 1] + ...  (left to right)
__global__ void k_row_sums(int n, const int* __restrict__ rp, const double* __restrict__ W,
                           const double* __restrict__ start, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = start[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc += W[k];
  out[i] = acc;
}

// lambda1 = max_i (D_i + sum_j W_ij); the bits of positive doubles order like
// unsigned integers, so the maximum is an integer atomic max.
__global__ void k_rowabs_max(int n, const int* __restrict__ rp, const double* __restrict__ W,
                             const double* __restrict__ D, unsigned long long* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    v = D[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) v += W[k];
  }
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

// ------------------------------------------------------------------ scan
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;

// Exclusive scan of tiles of 2048 values: in[i] for i < n_in, 0 beyond;
// writes out[i] for i < n_out and each tile's total.
__global__ void k_scan_tile(const int* __restrict__ in, int n_in, int* __restrict__ out, int n_out,
                            int* __restrict__ tile_sums) {
  __shared__ int wsum[TPB / 64];
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int t = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    v[q] = (base + q < n_in) ? in[base + q] : 0;
    t += v[q];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int incl = wave_incl_scan(t);
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += wsum[w];
  int run = woff + incl - t;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; ++q) {
    if (base + q < n_out) out[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == TPB - 1) tile_sums[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(int* out, int n, const int* __restrict__ tile_off) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / SCAN_TILE];
}

// out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
int32_t scan_excl(Temps& T, const int* in, int n, int* out, hipStream_t s) {
  const int n_out = n + 1;
  const int tiles = (n_out + SCAN_TILE - 1) / SCAN_TILE;
  int* sums = nullptr;
  AMG_TRY(T.get(&sums, tiles + 1));
  hipLaunchKernelGGL(k_scan_tile, dim3(tiles), dim3(TPB), 0, s, in, n, out, n_out, sums);
  AMG_HIP(hipGetLastError());
  if (tiles > 1) {
    int* off = nullptr;
    AMG_TRY(T.get(&off, tiles + 1));
    AMG_TRY(scan_excl(T, sums, tiles, off, s));
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n_out)), dim3(TPB), 0, s, out, n_out, off);
    AMG_HIP(hipGetLastError());
  }
  return AMG_OK;
}

int32_t read_int(const int* dptr, int* host, hipStream_t s) {
  AMG_HIP(hipMemcpyAsync(host, dptr, sizeof(int), hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

// ------------------------------------------------------------------ matching
// Strength of every stored entry, taken from the entry of row min(i, j) and
// mirrored to its partner so both endpoints see the same key.
__global__ void k_strength(int n, const int* __restrict__ rp, const int* __restrict__ col,
                           const double* __restrict__ W, const double* __restrict__ D, int raw,
                           double* __restrict__ S) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double Di = D[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = col[k];
    if (j < i) continue;
    const double w = W[k];
    double s;
    if (raw) {
      s = w;
    } else {
      const double ww = w * w;
      const double dd = Di * D[j];
      s = ww / dd;
    }
    S[k] = s;
    int lo = rp[j], hi = rp[j + 1];
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (col[mid] < i) lo = mid + 1; else hi = mid;
    }
    S[lo] = s;
  }
}

// Hash of an edge for hash tie-breaking: MurmurHash3's 32-bit finalizer of
// (a * 2654435761 + b) mod 2^32.
__device__ __forceinline__ uint32_t tie_hash(uint32_t a, uint32_t b) {
  uint32_t x = a * 2654435761u + b;
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// Edge order: (-s, [hash,] min endpoint, max endpoint) ascending.  True if
// edge 1 comes first.
__device__ __forceinline__ bool edge_first(double s1, int a1, int b1, double s2, int a2, int b2, bool hashed) {
  if (s1 != s2) return s1 > s2;
  if (hashed) {
    const uint32_t h1 = tie_hash((uint32_t)a1, (uint32_t)b1), h2 = tie_hash((uint32_t)a2, (uint32_t)b2);
    if (h1 != h2) return h1 < h2;
  }
  if (a1 != a2) return a1 < a2;
  return b1 < b2;
}

// mate[v]: -1 free, -2 finished single, >= 0 partner.  The neighbours are
// read in chunks of 8 (all column indices and strengths of a chunk, then all
// their mates) so that the loads of a chunk are in flight together; the best
// edge is a maximum in a strict order, so the scan order does not matter.
__device__ __forceinline__ int best_free_neighbour(int v, const int* __restrict__ rp, const int* __restrict__ col,
                                                   const double* __restrict__ S, const int* mate, bool hashed) {
  constexpr int U = 8;
  int best = -1, ba = 0, bb = 0;
  double bs = 0.0;
  const int k0 = rp[v], k1 = rp[v + 1];
  for (int k = k0; k < k1; k += U) {
    int u[U], mu[U];
    double sv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int kk = min(k + j, k1 - 1);
      u[j] = col[kk];
      sv[j] = S[kk];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) mu[j] = mate[u[j]];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      if (k + j >= k1 || mu[j] != -1) continue;
      const int a = u[j] < v ? u[j] : v, b = u[j] < v ? v : u[j];
      if (best < 0 || edge_first(sv[j], a, b, bs, ba, bb, hashed)) {
        best = u[j];
        bs = sv[j];
        ba = a;
        bb = b;
      }
    }
  }
  return best;
}

// ---- handshake matching on worklists
//
// Every free vertex points at its best free neighbour (cand); mutual pairs
// match, vertices with no free neighbour become singletons (mate = -2).  A
// free vertex's best free neighbour can only change when that neighbour
// leaves the free set (removing any other vertex does not change a maximum),
// so each round re-evaluates only the vertices whose candidate has just left
// it.  The proposals of every round are therefore those of the full
// handshake, and so is the result: the unique locally dominant matching,
// which is the greedy matching in the strict edge order.
//
// Round r: evaluate the list W_r (cand = best free neighbour or -2); accept
// (mutual pairs and singletons leave the free set, listed in `fresh`); push
// the free vertices whose candidate is in `fresh` onto W_{r+1}.  stamp[v] is
// the round of the list v was last put on (round 0 = every vertex).

// Appends v to list when `take`, one atomic per wavefront.
__device__ __forceinline__ void list_push(int* list, int* size, bool take, int v) {
  const unsigned long long m = __ballot(take);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(size, __popcll(m));
  base = __shfl(base, leader, 64);
  if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

struct MatchState {
  const int* rp;
  const int* col;
  const double* S;
  int* mate;
  int* cand;
  int* stamp;
  int* W[2];    // the round's list and the next one
  int* fresh;   // vertices that left the free set this round
  int* size;    // size[0], size[1]: |W[0]|, |W[1]|; size[2]: |fresh|; size[3]: rounds with work
  int hashed;   // hash tie-breaking
};

__device__ __forceinline__ void mw_eval_one(const MatchState& M, int v) {
  const int b = best_free_neighbour(v, M.rp, M.col, M.S, M.mate, M.hashed != 0);
  M.cand[v] = b >= 0 ? b : -2;
}

__device__ __forceinline__ void mw_accept_one(const MatchState& M, int v, int round, int* fresh, int* fsize,
                                              bool valid) {
  bool leave_v = false, leave_u = false;
  int u = -1;
  if (valid) {
    u = M.cand[v];
    if (u == -2) {
      M.mate[v] = -2;
      leave_v = true;
    } else if (M.cand[u] == v) {
      M.mate[v] = u;
      M.mate[u] = v;
      leave_v = true;
      leave_u = M.stamp[u] != round;  // a partner not on this round's list is listed by v
    }
  }
  list_push(fresh, fsize, leave_v, v);
  list_push(fresh, fsize, leave_u, u);
}

// neighbours in chunks of 8, as in best_free_neighbour
__device__ __forceinline__ void mw_push_one(const MatchState& M, int m, int next_round, int* W, int* wsize) {
  constexpr int U = 8;
  const int k0 = M.rp[m], k1 = M.rp[m + 1];
  for (int k = k0; k < k1; k += U) {
    int x[U], mx[U], cx[U];
#pragma unroll
    for (int j = 0; j < U; ++j) x[j] = M.col[min(k + j, k1 - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      mx[j] = M.mate[x[j]];
      cx[j] = M.cand[x[j]];
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const bool take = k + j < k1 && mx[j] == -1 && cx[j] == m;
      if (take) M.stamp[x[j]] = next_round;
      list_push(W, wsize, take, x[j]);
    }
  }
}

// Multi-block rounds (large lists): grid-stride over the list held on the
// device; `implicit_n` > 0 stands for the list 0..n-1 (round 0).
__global__ void __launch_bounds__(256) k_mw_eval(MatchState M, int cur, int implicit_n) {
  const int sz = implicit_n > 0 ? implicit_n : M.size[cur];
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) {
    M.size[cur ^ 1] = 0;
    M.size[2] = 0;
    if (sz > 0) M.size[3] += 1;
  }
  for (int i = g; i < sz; i += gridDim.x * blockDim.x) mw_eval_one(M, implicit_n > 0 ? i : M.W[cur][i]);
}

__global__ void __launch_bounds__(256) k_mw_accept(MatchState M, int cur, int implicit_n, int round) {
  const int sz = implicit_n > 0 ? implicit_n : M.size[cur];
  const int stride = gridDim.x * blockDim.x;
  // whole wavefronts iterate together (list_push needs the wavefront)
  const int lim = (sz + 63) & ~63;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += stride) {
    const bool valid = i < sz;
    const int v = valid ? (implicit_n > 0 ? i : M.W[cur][i]) : 0;
    mw_accept_one(M, v, round, M.fresh, &M.size[2], valid);
  }
}

__global__ void __launch_bounds__(256) k_mw_push(MatchState M, int cur, int round) {
  const int sz = M.size[2];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < sz; i += gridDim.x * blockDim.x)
    mw_push_one(M, M.fresh[i], round + 1, M.W[cur ^ 1], &M.size[cur ^ 1]);
}

// Rounds in one workgroup while the list is short: workgroup barriers
// instead of launches.  The counters live in LDS.  Stops when the list is
// empty, longer than `max_list`, or after `max_rounds` rounds; io[0] (round)
// and io[1] (current list) carry the position in and out.
__global__ void __launch_bounds__(1024) k_mw_small(MatchState M, int* io, int max_list, int max_rounds) {
  __shared__ int s_size[2], s_fresh, s_work;
  int round = io[0], cur = io[1];
  if (threadIdx.x == 0) {
    s_size[0] = M.size[0];
    s_size[1] = M.size[1];
    s_work = M.size[3];
  }
  __syncthreads();
  for (int it = 0; it < max_rounds; ++it) {
    const int sz = s_size[cur];
    if (sz == 0 || sz > max_list) break;  // uniform: read after a barrier
    for (int i = threadIdx.x; i < sz; i += blockDim.x) mw_eval_one(M, M.W[cur][i]);
    if (threadIdx.x == 0) {
      s_size[cur ^ 1] = 0;
      s_fresh = 0;
      s_work += 1;
    }
    __syncthreads();
    const int lim = (sz + 63) & ~63;
    for (int i = threadIdx.x; i < lim; i += blockDim.x) {
      const bool valid = i < sz;
      mw_accept_one(M, valid ? M.W[cur][i] : 0, round, M.fresh, &s_fresh, valid);
    }
    __syncthreads();
    const int nf = s_fresh;
    for (int i = threadIdx.x; i < nf; i += blockDim.x) mw_push_one(M, M.fresh[i], round + 1, M.W[cur ^ 1], &s_size[cur ^ 1]);
    __syncthreads();
    cur ^= 1;
    ++round;
  }
  if (threadIdx.x == 0) {
    M.size[0] = s_size[0];
    M.size[1] = s_size[1];
    M.size[3] = s_work;
    io[0] = round;
    io[1] = cur;
  }
}

// ------------------------------------------------------------------ coarse numbering
__global__ void k_rep_flags(int n, const int* __restrict__ mate, int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = mate[i];
  flag[i] = (m < 0 || i < m) ? 1 : 0;
}

__global__ void k_pair_ids(int n, const int* __restrict__ mate, const int* __restrict__ pos,
                           int* __restrict__ ids, int* __restrict__ rep) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = mate[i];
  const int r = (m >= 0 && m < i) ? m : i;
  ids[i] = pos[r];
  if (r == i) rep[pos[i]] = i;
}

// ------------------------------------------------------------------ Galerkin (pairs)
__device__ __forceinline__ int partner(const int* mate, int a) {
  const int b = mate[a];
  return b >= 0 ? b : -1;
}

__global__ void k_gal_len(int nc, const int* __restrict__ rep, const int* __restrict__ mate,
                          const int* __restrict__ rp, int* __restrict__ len) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int a = rep[I], b = partner(mate, a);
  len[I] = (rp[a + 1] - rp[a]) + (b >= 0 ? rp[b + 1] - rp[b] : 0);
}

// For coarse row I = {a, b} (a < b): the pairs (J = agg(j), w) of rows a then b
// with J != I, stably sorted by J (insertion sort: equal keys keep the fine
// order), and the number of distinct J.
__global__ void k_gal_sort(int nc, const int* __restrict__ rep, const int* __restrict__ mate,
                           const int* __restrict__ rp, const int* __restrict__ col,
                           const double* __restrict__ W, const int* __restrict__ ids,
                           const int* __restrict__ toff, int* __restrict__ tJ, double* __restrict__ tW,
                           int* __restrict__ tcnt, int* __restrict__ ucnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int a = rep[I], b = partner(mate, a);
  const int o = toff[I];
  int cnt = 0;
  for (int t = 0; t < 2; ++t) {
    const int row = t == 0 ? a : b;
    if (row < 0) break;
    for (int k = rp[row]; k < rp[row + 1]; ++k) {
      const int J = ids[col[k]];
      if (J == I) continue;
      const double w = W[k];
      int p = cnt;
      while (p > 0 && tJ[o + p - 1] > J) {
        tJ[o + p] = tJ[o + p - 1];
        tW[o + p] = tW[o + p - 1];
        --p;
      }
      tJ[o + p] = J;
      tW[o + p] = w;
      ++cnt;
    }
  }
  int u = 0;
  for (int q = 0; q < cnt; ++q) u += (q == 0 || tJ[o + q] != tJ[o + q - 1]);
  tcnt[I] = cnt;
  ucnt[I] = u;
}

// Sum every run of equal J left to right; coarse d_H = d_a (+ d_b).
__global__ void k_gal_reduce(int nc, const int* __restrict__ toff, const int* __restrict__ tcnt,
                             const int* __restrict__ tJ, const double* __restrict__ tW,
                             const int* __restrict__ rpH, int* __restrict__ colH, double* __restrict__ WH,
                             const int* __restrict__ rep, const int* __restrict__ mate,
                             const double* __restrict__ d, double* __restrict__ dH) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int o = toff[I], cnt = tcnt[I];
  int out = rpH[I] - 1;
  int lastJ = -1;
  double acc = 0.0;
  for (int q = 0; q < cnt; ++q) {
    const int J = tJ[o + q];
    if (J != lastJ) {
      if (out >= rpH[I]) WH[out] = acc;
      ++out;
      colH[out] = J;
      acc = tW[o + q];
      lastJ = J;
    } else {
      acc += tW[o + q];
    }
  }
  if (cnt > 0) WH[out] = acc;
  const int a = rep[I], b = partner(mate, a);
  double dd = d[a];
  if (b >= 0) dd += d[b];
  dH[I] = dd;
}

__global__ void k_compose(int n, int* __restrict__ agg, const int* __restrict__ ids) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) agg[i] = ids[agg[i]];
}

// ------------------------------------------------------------------ member lists
__global__ void k_count(int n, const int* __restrict__ agg, int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[agg[i]], 1);
}

__global__ void k_scatter_members(int n, const int* __restrict__ agg, const int* __restrict__ off,
                                  int* cursor, int* __restrict__ members) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = agg[i];
  members[off[a] + atomicAdd(&cursor[a], 1)] = i;
}

// Members of each aggregate in increasing vertex order (deterministic; the
// keys are distinct).  Insertion sort for the small aggregates of matching,
// heapsort for the large ones an independent set of the graph of A^k can make.
__device__ void sift_down(int* a, int root, int m) {
  const int v = a[root];
  int r = root;
  for (;;) {
    int c = 2 * r + 1;
    if (c >= m) break;
    if (c + 1 < m && a[c + 1] > a[c]) ++c;
    if (a[c] <= v) break;
    a[r] = a[c];
    r = c;
  }
  a[r] = v;
}

__global__ void k_sort_members(int nc, const int* __restrict__ off, int* __restrict__ members) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int o = off[I], e = off[I + 1], m = e - o;
  if (m > 32) {
    int* a = members + o;
    for (int r = m / 2 - 1; r >= 0; --r) sift_down(a, r, m);
    for (int k = m - 1; k > 0; --k) {
      const int t = a[0];
      a[0] = a[k];
      a[k] = t;
      sift_down(a, 0, k);
    }
    return;
  }
  for (int k = o + 1; k < e; ++k) {
    const int v = members[k];
    int p = k;
    while (p > o && members[p - 1] > v) {
      members[p] = members[p - 1];
      --p;
    }
    members[p] = v;
  }
}

// ------------------------------------------------------------------ MIS aggregation
// Section 2's partitioning as the paper's experiments use it: (A) a maximal
// independent set S of the graph of A^k, (B) every vertex joins its nearest
// vertex of S.  S is the greedy set in decreasing priority key(v) =
// splitmix64(v), computed in rounds: an undecided vertex joins when no member
// of S and no undecided vertex of larger key lies within distance k (k hops of
// max / or propagation), and leaves when a member lies within distance k --
// the same set as taking the vertices one by one in key order.
__device__ __forceinline__ unsigned long long mis_key(int v) { return splitmix64((uint64_t)v); }

// state: 0 undecided, 1 in S, 2 out
__global__ void k_mis_seed(int n, const int* __restrict__ state, unsigned long long* __restrict__ mx,
                           int* __restrict__ near) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  mx[v] = state[v] == 0 ? mis_key(v) : 0ull;
  near[v] = state[v] == 1 ? 1 : 0;
}

// one hop over the closed neighbourhood: the largest undecided key and
// whether a member of S is there
__global__ void k_mis_hop(int n, const int* __restrict__ rp, const int* __restrict__ col,
                          const unsigned long long* __restrict__ mx_in, const int* __restrict__ near_in,
                          unsigned long long* __restrict__ mx_out, int* __restrict__ near_out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  unsigned long long m = mx_in[v];
  int f = near_in[v];
  for (int e = rp[v]; e < rp[v + 1]; ++e) {
    const int u = col[e];
    const unsigned long long mu = mx_in[u];
    m = mu > m ? mu : m;
    f |= near_in[u];
  }
  mx_out[v] = m;
  near_out[v] = f;
}

__global__ void k_mis_decide(int n, int* __restrict__ state, const unsigned long long* __restrict__ mx,
                             const int* __restrict__ near, int* undecided) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || state[v] != 0) return;
  if (near[v]) {
    state[v] = 2;
  } else if (mx[v] == mis_key(v)) {
    state[v] = 1;
  } else {
    atomicAdd(undecided, 1);
  }
}

__global__ void k_owner_init(int n, const int* __restrict__ state, int* __restrict__ owner, int* __restrict__ flag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  owner[v] = state[v] == 1 ? v : -1;
  flag[v] = state[v] == 1 ? 1 : 0;
}

// one breadth-first hop from all of S: a vertex first reached now takes the
// smallest owner among its reached neighbours (all reached one hop earlier)
__global__ void k_owner_hop(int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const int* __restrict__ own_in, int* __restrict__ own_out, int* changed) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int o = own_in[v];
  if (o < 0) {
    int best = INT_MAX;
    for (int e = rp[v]; e < rp[v + 1]; ++e) {
      const int ou = own_in[col[e]];
      if (ou >= 0 && ou < best) best = ou;
    }
    if (best != INT_MAX) {
      o = best;
      *changed = 1;
    }
  }
  own_out[v] = o;
}

__global__ void k_owner_ids(int n, const int* __restrict__ owner, const int* __restrict__ pos, int* __restrict__ ids,
                            int* bad) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int o = owner[v];
  if (o < 0) {
    ids[v] = 0;
    atomicAdd(bad, 1);
  } else {
    ids[v] = pos[o];
  }
}

// Galerkin over member lists: coarse row I gathers the entries of its member
// rows (members in increasing order, entries in row order), drops J = I,
// sorts by J keeping that order among equal J (insertion), and adds runs of
// equal J left to right -- the sums of the sequential definition.
__global__ void k_galm_len(int nc, const int* __restrict__ moff, const int* __restrict__ members,
                           const int* __restrict__ rp, int* __restrict__ len) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int s = 0;
  for (int k = moff[I]; k < moff[I + 1]; ++k) {
    const int i = members[k];
    s += rp[i + 1] - rp[i];
  }
  len[I] = s;
}

__global__ void k_galm_sort(int nc, const int* __restrict__ moff, const int* __restrict__ members,
                            const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ W,
                            const int* __restrict__ ids, const int* __restrict__ toff, int* __restrict__ tJ,
                            double* __restrict__ tW, int* __restrict__ tcnt, int* __restrict__ ucnt,
                            int max_len) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int o = toff[I];
  if (toff[I + 1] - o > max_len) return;  // a long row: the hash kernel's
  int c = 0;
  for (int k = moff[I]; k < moff[I + 1]; ++k) {
    const int i = members[k];
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int J = ids[col[e]];
      if (J == I) continue;
      const double w = W[e];
      int p = o + c;
      while (p > o && tJ[p - 1] > J) {
        tJ[p] = tJ[p - 1];
        tW[p] = tW[p - 1];
        --p;
      }
      tJ[p] = J;
      tW[p] = w;
      ++c;
    }
  }
  int u = 0;
  for (int p = 0; p < c; ++p)
    if (p == 0 || tJ[o + p] != tJ[o + p - 1]) ++u;
  tcnt[I] = c;
  ucnt[I] = u;
}

__global__ void k_galm_reduce(int nc, const int* __restrict__ toff, const int* __restrict__ tcnt,
                              const int* __restrict__ tJ, const double* __restrict__ tW, const int* __restrict__ crp,
                              int* __restrict__ ccol, double* __restrict__ cW, const int* __restrict__ moff,
                              const int* __restrict__ members, const double* __restrict__ d, double* __restrict__ cd) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int o = toff[I], c = tcnt[I];
  int q = crp[I];
  int p = 0;
  while (p < c) {
    const int J = tJ[o + p];
    double s = 0.0;
    while (p < c && tJ[o + p] == J) {
      s += tW[o + p];
      ++p;
    }
    ccol[q] = J;
    cW[q] = s;
    ++q;
  }
  double dd = 0.0;
  for (int k = moff[I]; k < moff[I + 1]; ++k) dd += d[members[k]];
  cd[I] = dd;
}

// The same coarse rows for long rows (more than kGalHashLen gathered entries;
// the insertion sort above is quadratic in the row), in time linear in the
// row: one wavefront per coarse row visits its entries in the sequential order
// (members in increasing index, entries in row order), 64 at a time; lane 0
// adds each weight to its coarse column's slot of an LDS hash table (a slot
// starts at 0 and adds in that order: the sums of the sequential definition);
// the distinct columns are then written in increasing order with their sums,
// one entry per column, which k_galm_reduce copies unchanged.  A row with more
// than kGalFill distinct columns sets *overflow, and the caller then sorts
// every row instead.
constexpr int kGalHashLen = 384, kGalTable = 1024, kGalFill = 768;

__global__ void __launch_bounds__(64) k_galm_hash(int nc, const int* __restrict__ moff,
                                                  const int* __restrict__ members, const int* __restrict__ rp,
                                                  const int* __restrict__ col, const double* __restrict__ W,
                                                  const int* __restrict__ ids, const int* __restrict__ toff,
                                                  int* __restrict__ tJ, double* __restrict__ tW,
                                                  int* __restrict__ tcnt, int* __restrict__ ucnt, int* overflow) {
  __shared__ int key[kGalTable];
  __shared__ double sum[kGalTable];
  __shared__ int dk[kGalFill];
  __shared__ double dsum[kGalFill];
  __shared__ int cj[64];
  __shared__ double cw[64];
  __shared__ int nd_s, ovf_s, nk_s;
  const int I = blockIdx.x;
  const int lane = threadIdx.x;
  if (I >= nc || toff[I + 1] - toff[I] <= kGalHashLen) return;
  for (int s = lane; s < kGalTable; s += 64) key[s] = -1;
  if (lane == 0) {
    nd_s = 0;
    ovf_s = 0;
    nk_s = 0;
  }
  __syncthreads();
  const int m1 = moff[I + 1];
  for (int m = moff[I]; m < m1; ++m) {
    const int i = members[m];
    const int e1 = rp[i + 1];
    for (int e0 = rp[i]; e0 < e1; e0 += 64) {
      const int cnt = min(64, e1 - e0);
      if (lane < cnt) {
        cj[lane] = ids[col[e0 + lane]];
        cw[lane] = W[e0 + lane];
      }
      __syncthreads();
      if (lane == 0) {
        for (int t = 0; t < cnt; ++t) {
          const int J = cj[t];
          if (J == I) continue;
          int s = (int)(((unsigned)J * 2654435761u) & (unsigned)(kGalTable - 1));
          while (key[s] != -1 && key[s] != J) s = (s + 1) & (kGalTable - 1);
          if (key[s] == -1) {
            if (nd_s == kGalFill) {
              ovf_s = 1;
              break;
            }
            key[s] = J;
            sum[s] = 0.0;
            ++nd_s;
          }
          sum[s] += cw[t];
        }
      }
      __syncthreads();
      if (ovf_s) break;
    }
    if (ovf_s) break;
  }
  if (ovf_s) {
    if (lane == 0) atomicOr(overflow, 1);
    return;
  }
  for (int s = lane; s < kGalTable; s += 64) {
    const int J = key[s];
    if (J >= 0) {
      const int q = atomicAdd(&nk_s, 1);
      dk[q] = J;
      dsum[q] = sum[s];
    }
  }
  __syncthreads();
  const int nd = nd_s, o = toff[I];
  for (int q = lane; q < nd; q += 64) {
    const int J = dk[q];
    int rank = 0;
    for (int t = 0; t < nd; ++t) rank += dk[t] < J;
    tJ[o + rank] = J;
    tW[o + rank] = dsum[q];
  }
  if (lane == 0) {
    tcnt[I] = nd;
    ucnt[I] = nd;
  }
}

// ------------------------------------------------------------------ sliced ELL
// Row order of a sorted layout: inside each group of 64 rows (the rows one
// wavefront covers), rows by decreasing length, ties by index.  A wavefront
// then still touches the same vector cache lines as in row order.
__global__ void __launch_bounds__(256) k_sell_perm(int n, const int* __restrict__ rp, int* __restrict__ perm) {
  __shared__ int deg[256];
  const int i = threadIdx.x, r = blockIdx.x * 256 + i;
  const int di = r < n ? rp[r + 1] - rp[r] : -1;
  deg[i] = di;
  __syncthreads();
  if (r >= n) return;
  const int g0 = i & ~63;
  int rank = 0;
  for (int k = g0; k < g0 + 64; ++k) {
    const int dk = deg[k];
    rank += (dk > di) || (dk == di && k < i);
  }
  perm[blockIdx.x * 256 + g0 + rank] = r;
}

__device__ __forceinline__ int sell_row(int q, int n, const int* __restrict__ perm) {
  return q < n ? (perm ? perm[q] : q) : -1;
}

// Steps per slice: the longest row of the slice, in units of K entries.
__global__ void k_sell_width(int nslots, int n, const int* __restrict__ rp, const int* __restrict__ perm, int lc,
                             int lk, int* __restrict__ w) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = sell_row(q, n, perm);
  int deg = r >= 0 ? rp[r + 1] - rp[r] : 0;
  for (int off = (1 << lc) >> 1; off > 0; off >>= 1) {
    const int o = __shfl_xor(deg, off, 64);
    deg = o > deg ? o : deg;
  }
  if (q < nslots && (q & ((1 << lc) - 1)) == 0) w[q >> lc] = (deg + (1 << lk) - 1) >> lk;
}

__global__ void k_sell_len(int ns, const int* __restrict__ w, int shift, int* __restrict__ len) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns) len[s] = w[s] << shift;
}

// Either weight array may be null (not wanted).
__global__ void k_sell_fill(int nslots, int n, const int* __restrict__ rp, const int* __restrict__ col,
                            const double* __restrict__ W, const int* __restrict__ perm, int lc, int lk,
                            const int* __restrict__ off, const int* __restrict__ width, int* __restrict__ scol,
                            double* __restrict__ sval, float* __restrict__ svalf) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslots) return;
  const int r = sell_row(q, n, perm);
  const int s = q >> lc, p = q & ((1 << lc) - 1), K = 1 << lk;
  const int wd = width[s], stride = K << lc;
  const int b = r >= 0 ? rp[r] : 0;
  const int deg = r >= 0 ? rp[r + 1] - b : 0;
  const int self = r >= 0 ? r : 0;
  for (int t = 0; t < wd; ++t) {
    for (int j = 0; j < K; ++j) {
      const int k = t * K + j;
      const int idx = off[s] + t * stride + p * K + j;
      int c = self;
      double v = 0.0;
      if (k < deg) {
        c = col[b + k];
        v = W[b + k];
      }
      scol[idx] = c;
      if (sval) sval[idx] = v;
      if (svalf) svalf[idx] = (float)v;
    }
  }
}

__global__ void k_to_float(int n, const double* __restrict__ a, float* __restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// ------------------------------------------------------------------ coarsest level
__global__ void k_dense(int n, const int* __restrict__ rp, const int* __restrict__ col,
                        const double* __restrict__ W, const double* __restrict__ D, double* __restrict__ A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  A[(size_t)i * n + i] = D[i];
  for (int k = rp[i]; k < rp[i + 1]; ++k) A[(size_t)i * n + col[k]] = -W[k];
}

// A + c 1 1^T on the dense n x n coarsest matrix
__global__ void k_add_const(size_t nn, double* __restrict__ A, double c) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) A[i] = A[i] + c;
}

// Right-looking Cholesky A = L L^T in one workgroup (row-major, lower part);
// the strict upper triangle is zeroed.  status = 1 on a non-positive pivot.
__global__ void __launch_bounds__(1024) k_chol(int n, double* A, int* status) {
  __shared__ double piv;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const double akk = A[(size_t)k * n + k];
      if (!(akk > 0.0) || !isfinite(akk)) bad = 1;
      piv = sqrt(akk);
      A[(size_t)k * n + k] = piv;
    }
    __syncthreads();
    if (bad) break;
    const double p = piv;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[(size_t)i * n + k] /= p;
    __syncthreads();
    const int m = n - k - 1;
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
      const int i = k + 1 + t / m, j = k + 1 + t % m;
      if (j <= i) A[(size_t)i * n + j] -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t % n;
    if (j > i) A[t] = 0.0;
  }
  if (threadIdx.x == 0) *status = bad;
}

// Inverse of the lower Cholesky factor: thread j computes column j of L^-1 by
// forward substitution (n <= 1024, one workgroup); also writes the transpose.
__global__ void __launch_bounds__(1024) k_tri_inv(int n, const double* __restrict__ L, double* __restrict__ X,
                                                  double* __restrict__ XT) {
  const int j = threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < n; ++i) {
    double v = 0.0;
    if (i >= j) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= L[(size_t)i * n + k] * X[(size_t)k * n + j];
      v = acc / L[(size_t)i * n + i];
    }
    X[(size_t)i * n + j] = v;
    XT[(size_t)j * n + i] = v;
  }
}

// ------------------------------------------------------------------ host helpers
using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

struct Graph {  // a pass graph on the device (not owned)
  int n = 0;
  int nnz = 0;
  int* rp = nullptr;
  int* col = nullptr;
  double* W = nullptr;
  double* d = nullptr;
  double* D = nullptr;
};

// One matching pass on g: mate[] (device) and the number of rounds.
int32_t match_pass(Temps& T, const Graph& g, int raw, int hashed, int* mate, int* rounds, hipStream_t s) {
  double* S = nullptr;
  int *cand = nullptr, *stamp = nullptr, *w0 = nullptr, *w1 = nullptr, *fresh = nullptr, *size = nullptr,
      *io = nullptr;
  AMG_TRY(T.get(&S, std::max(g.nnz, 1)));
  AMG_TRY(T.get(&cand, g.n));
  AMG_TRY(T.get(&stamp, g.n));
  AMG_TRY(T.get(&w0, g.n));
  AMG_TRY(T.get(&w1, g.n));
  AMG_TRY(T.get(&fresh, g.n));
  AMG_TRY(T.get(&size, 4));
  AMG_TRY(T.get(&io, 2));
  hipLaunchKernelGGL(k_strength, dim3(nblk(g.n)), dim3(TPB), 0, s, g.n, g.rp, g.col, g.W, g.D, raw, S);
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(g.n)), dim3(TPB), 0, s, (size_t)g.n, mate, -1);
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(g.n)), dim3(TPB), 0, s, (size_t)g.n, stamp, 0);
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)4, size, 0);
  AMG_HIP(hipGetLastError());
  const MatchState M{g.rp, g.col, S, mate, cand, stamp, {w0, w1}, fresh, size, hashed};
  // lists up to this long run in one workgroup; multi-block rounds otherwise
  constexpr int kSmallList = 4096, kBatch = 8, kSmallRounds = 4096;
  const int grid = std::min(nblk(g.n), 2048);
  int round = 0, cur = 0;
  if (g.n <= kSmallList) {
    hipLaunchKernelGGL(k_iota, dim3(nblk(g.n)), dim3(TPB), 0, s, g.n, w0);
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)1, size, g.n);
  } else {
    // round 0: every vertex
    hipLaunchKernelGGL(k_mw_eval, dim3(grid), dim3(256), 0, s, M, cur, g.n);
    hipLaunchKernelGGL(k_mw_accept, dim3(grid), dim3(256), 0, s, M, cur, g.n, round);
    hipLaunchKernelGGL(k_mw_push, dim3(grid), dim3(256), 0, s, M, cur, round);
    cur ^= 1;
    ++round;
  }
  AMG_HIP(hipGetLastError());
  for (;;) {
    int h[4];
    AMG_HIP(hipMemcpyAsync(h, size, sizeof(h), hipMemcpyDeviceToHost, s));
    AMG_HIP(hipStreamSynchronize(s));
    if (h[cur] == 0) {
      *rounds = h[3];
      break;
    }
    if (round > 4 * g.n + 64) {
      set_last_error("matching did not terminate");
      return AMG_ERR_DEVICE;
    }
    if (h[cur] <= kSmallList) {
      const int hio[2] = {round, cur};
      AMG_HIP(hipMemcpyAsync(io, hio, sizeof(hio), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_mw_small, dim3(1), dim3(1024), 0, s, M, io, kSmallList, kSmallRounds);
      AMG_HIP(hipGetLastError());
      int oio[2];
      AMG_HIP(hipMemcpyAsync(oio, io, sizeof(oio), hipMemcpyDeviceToHost, s));
      AMG_HIP(hipStreamSynchronize(s));
      round = oio[0];
      cur = oio[1];
      continue;
    }
    for (int b = 0; b < kBatch; ++b, ++round, cur ^= 1) {
      hipLaunchKernelGGL(k_mw_eval, dim3(grid), dim3(256), 0, s, M, cur, 0);
      hipLaunchKernelGGL(k_mw_accept, dim3(grid), dim3(256), 0, s, M, cur, 0, round);
      hipLaunchKernelGGL(k_mw_push, dim3(grid), dim3(256), 0, s, M, cur, round);
    }
    AMG_HIP(hipGetLastError());
  }
  return AMG_OK;
}

// Coarse numbering and Galerkin operator of one pass.  Allocates the coarse
// graph from `alloc_owned` (hierarchy-owned) or from T.
int32_t galerkin_pass(amg_hier* h, Temps& T, const Graph& g, const int* mate, bool owned, Graph* out,
                      int** ids_out, double* t_agg_ms, double* t_gal_ms, hipStream_t s) {
  auto t0 = clk::now();
  int *flag, *pos, *ids, *rep;
  AMG_TRY(T.get(&flag, g.n));
  AMG_TRY(T.get(&pos, g.n + 1));
  AMG_TRY(T.get(&ids, g.n));
  hipLaunchKernelGGL(k_rep_flags, dim3(nblk(g.n)), dim3(TPB), 0, s, g.n, mate, flag);
  AMG_TRY(scan_excl(T, flag, g.n, pos, s));
  int nc = 0;
  AMG_TRY(read_int(pos + g.n, &nc, s));
  AMG_TRY(T.get(&rep, nc));
  hipLaunchKernelGGL(k_pair_ids, dim3(nblk(g.n)), dim3(TPB), 0, s, g.n, mate, pos, ids, rep);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  *t_agg_ms += ms_since(t0);

  auto t1 = clk::now();
  int *len, *toff, *tJ, *tcnt, *ucnt;
  double* tW;
  AMG_TRY(T.get(&len, nc));
  AMG_TRY(T.get(&toff, nc + 1));
  AMG_TRY(T.get(&tJ, std::max(g.nnz, 1)));
  AMG_TRY(T.get(&tW, std::max(g.nnz, 1)));
  AMG_TRY(T.get(&tcnt, nc));
  AMG_TRY(T.get(&ucnt, nc));
  hipLaunchKernelGGL(k_gal_len, dim3(nblk(nc)), dim3(TPB), 0, s, nc, rep, mate, g.rp, len);
  AMG_TRY(scan_excl(T, len, nc, toff, s));
  hipLaunchKernelGGL(k_gal_sort, dim3(nblk(nc)), dim3(TPB), 0, s, nc, rep, mate, g.rp, g.col, g.W, ids,
                     toff, tJ, tW, tcnt, ucnt);
  Graph c;
  c.n = nc;
  if (owned) {
    AMG_TRY(dalloc(h, &c.rp, nc + 1));
  } else {
    AMG_TRY(T.get(&c.rp, nc + 1));
  }
  AMG_TRY(scan_excl(T, ucnt, nc, c.rp, s));
  AMG_TRY(read_int(c.rp + nc, &c.nnz, s));
  if (owned) {
    AMG_TRY(dalloc(h, &c.col, std::max(c.nnz, 1)));
    AMG_TRY(dalloc(h, &c.W, std::max(c.nnz, 1)));
    AMG_TRY(dalloc(h, &c.d, nc));
    AMG_TRY(dalloc(h, &c.D, nc));
  } else {
    AMG_TRY(T.get(&c.col, std::max(c.nnz, 1)));
    AMG_TRY(T.get(&c.W, std::max(c.nnz, 1)));
    AMG_TRY(T.get(&c.d, nc));
    AMG_TRY(T.get(&c.D, nc));
  }
  hipLaunchKernelGGL(k_gal_reduce, dim3(nblk(nc)), dim3(TPB), 0, s, nc, toff, tcnt, tJ, tW, c.rp, c.col, c.W,
                     rep, mate, g.d, c.d);
  hipLaunchKernelGGL(k_row_sums, dim3(nblk(nc)), dim3(TPB), 0, s, nc, c.rp, c.W, c.d, c.D);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  *t_gal_ms += ms_since(t1);
  *out = c;
  *ids_out = ids;
  return AMG_OK;
}

// One MIS aggregation of g (steps A and B): the aggregate map agg_out (n,
// hierarchy-owned) and the Galerkin coarse graph (hierarchy-owned).
int32_t mis_level(amg_hier* h, Temps& T, const Graph& g, int k, int** agg_out, Graph* out, int* rounds_out,
                  double* t_agg_ms, double* t_gal_ms, hipStream_t s) {
  auto t0 = clk::now();
  const int n = g.n;
  int *state, *nearA, *nearB, *counter, *ownA, *ownB, *flag, *pos, *ids;
  unsigned long long *mxA, *mxB;
  AMG_TRY(T.get(&state, n));
  AMG_TRY(T.get(&nearA, n));
  AMG_TRY(T.get(&nearB, n));
  AMG_TRY(T.get(&mxA, n));
  AMG_TRY(T.get(&mxB, n));
  AMG_TRY(T.get(&counter, 1));
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(n)), dim3(TPB), 0, s, (size_t)n, state, 0);
  AMG_HIP(hipGetLastError());
  int rounds = 0;
  for (;;) {
    if (rounds > n + 1) {
      set_last_error("independent set rounds did not terminate");
      return AMG_ERR_DEVICE;
    }
    ++rounds;
    hipLaunchKernelGGL(k_mis_seed, dim3(nblk(n)), dim3(TPB), 0, s, n, state, mxA, nearA);
    unsigned long long *mi = mxA, *mo = mxB;
    int *ni = nearA, *no = nearB;
    for (int hop = 0; hop < k; ++hop) {
      hipLaunchKernelGGL(k_mis_hop, dim3(nblk(n)), dim3(TPB), 0, s, n, g.rp, g.col, mi, ni, mo, no);
      std::swap(mi, mo);
      std::swap(ni, no);
    }
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)1, counter, 0);
    hipLaunchKernelGGL(k_mis_decide, dim3(nblk(n)), dim3(TPB), 0, s, n, state, mi, ni, counter);
    AMG_HIP(hipGetLastError());
    int left = 0;
    AMG_TRY(read_int(counter, &left, s));
    if (left == 0) break;
  }
  // step B: breadth-first from the set
  AMG_TRY(T.get(&ownA, n));
  AMG_TRY(T.get(&ownB, n));
  AMG_TRY(T.get(&flag, n));
  AMG_TRY(T.get(&pos, n + 1));
  hipLaunchKernelGGL(k_owner_init, dim3(nblk(n)), dim3(TPB), 0, s, n, state, ownA, flag);
  AMG_HIP(hipGetLastError());
  for (int hop = 0;; ++hop) {
    if (hop > n + 1) {
      set_last_error("aggregate collection did not terminate");
      return AMG_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)1, counter, 0);
    hipLaunchKernelGGL(k_owner_hop, dim3(nblk(n)), dim3(TPB), 0, s, n, g.rp, g.col, ownA, ownB, counter);
    AMG_HIP(hipGetLastError());
    std::swap(ownA, ownB);
    int changed = 0;
    AMG_TRY(read_int(counter, &changed, s));
    if (!changed) break;
  }
  AMG_TRY(scan_excl(T, flag, n, pos, s));
  int nc = 0;
  AMG_TRY(read_int(pos + n, &nc, s));
  AMG_TRY(dalloc(h, &ids, n));
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)1, counter, 0);
  hipLaunchKernelGGL(k_owner_ids, dim3(nblk(n)), dim3(TPB), 0, s, n, ownA, pos, ids, counter);
  AMG_HIP(hipGetLastError());
  int bad = 0;
  AMG_TRY(read_int(counter, &bad, s));
  if (bad || nc < 1) {
    set_last_error("a vertex was not reached from the independent set (disconnected level)");
    return AMG_ERR_DISCONNECTED;
  }
  // member lists (increasing vertex order)
  int *cnt, *cursor, *moff, *members;
  AMG_TRY(T.get(&cnt, nc));
  AMG_TRY(T.get(&cursor, nc));
  AMG_TRY(T.get(&moff, nc + 1));
  AMG_TRY(T.get(&members, n));
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(nc)), dim3(TPB), 0, s, (size_t)nc, cnt, 0);
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(nc)), dim3(TPB), 0, s, (size_t)nc, cursor, 0);
  hipLaunchKernelGGL(k_count, dim3(nblk(n)), dim3(TPB), 0, s, n, ids, cnt);
  AMG_TRY(scan_excl(T, cnt, nc, moff, s));
  hipLaunchKernelGGL(k_scatter_members, dim3(nblk(n)), dim3(TPB), 0, s, n, ids, moff, cursor, members);
  hipLaunchKernelGGL(k_sort_members, dim3(nblk(nc)), dim3(TPB), 0, s, nc, moff, members);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  *t_agg_ms += ms_since(t0);

  auto t1 = clk::now();
  int *len, *toff, *tJ, *tcnt, *ucnt;
  double* tW;
  AMG_TRY(T.get(&len, nc));
  AMG_TRY(T.get(&toff, nc + 1));
  AMG_TRY(T.get(&tJ, std::max(g.nnz, 1)));
  AMG_TRY(T.get(&tW, std::max(g.nnz, 1)));
  AMG_TRY(T.get(&tcnt, nc));
  AMG_TRY(T.get(&ucnt, nc));
  hipLaunchKernelGGL(k_galm_len, dim3(nblk(nc)), dim3(TPB), 0, s, nc, moff, members, g.rp, len);
  AMG_TRY(scan_excl(T, len, nc, toff, s));
  int* overflow = nullptr;
  AMG_TRY(T.get(&overflow, 1));
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, (size_t)1, overflow, 0);
  // rows up to kGalHashLen entries: insertion sort, one thread per row; longer
  // rows: the hash kernel (all rows sorted if one has too many columns)
  hipLaunchKernelGGL(k_galm_sort, dim3(nblk(nc)), dim3(TPB), 0, s, nc, moff, members, g.rp, g.col, g.W, ids, toff, tJ,
                     tW, tcnt, ucnt, kGalHashLen);
  hipLaunchKernelGGL(k_galm_hash, dim3(nc), dim3(64), 0, s, nc, moff, members, g.rp, g.col, g.W, ids, toff, tJ, tW,
                     tcnt, ucnt, overflow);
  AMG_HIP(hipGetLastError());
  int overflowed = 0;
  AMG_TRY(read_int(overflow, &overflowed, s));
  if (overflowed) {
    hipLaunchKernelGGL(k_galm_sort, dim3(nblk(nc)), dim3(TPB), 0, s, nc, moff, members, g.rp, g.col, g.W, ids, toff,
                       tJ, tW, tcnt, ucnt, INT_MAX);
  }
  Graph c;
  c.n = nc;
  AMG_TRY(dalloc(h, &c.rp, nc + 1));
  AMG_TRY(scan_excl(T, ucnt, nc, c.rp, s));
  AMG_TRY(read_int(c.rp + nc, &c.nnz, s));
  AMG_TRY(dalloc(h, &c.col, std::max(c.nnz, 1)));
  AMG_TRY(dalloc(h, &c.W, std::max(c.nnz, 1)));
  AMG_TRY(dalloc(h, &c.d, nc));
  AMG_TRY(dalloc(h, &c.D, nc));
  hipLaunchKernelGGL(k_galm_reduce, dim3(nblk(nc)), dim3(TPB), 0, s, nc, toff, tcnt, tJ, tW, c.rp, c.col, c.W, moff,
                     members, g.d, c.d);
  hipLaunchKernelGGL(k_row_sums, dim3(nblk(nc)), dim3(TPB), 0, s, nc, c.rp, c.W, c.d, c.D);
  AMG_HIP(hipGetLastError());
  AMG_HIP(hipStreamSynchronize(s));
  *t_gal_ms += ms_since(t1);
  *out = c;
  *agg_out = ids;
  *rounds_out = rounds;
  return AMG_OK;
}

int32_t build_members(amg_hier* h, Temps& T, Level& lv, int nc, hipStream_t s) {
  int *cnt, *cursor;
  AMG_TRY(T.get(&cnt, nc));
  AMG_TRY(T.get(&cursor, nc));
  AMG_TRY(dalloc(h, &lv.members, lv.n));
  AMG_TRY(dalloc(h, &lv.member_off, nc + 1));
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(nc)), dim3(TPB), 0, s, (size_t)nc, cnt, 0);
  hipLaunchKernelGGL(k_fill<int>, dim3(nblk(nc)), dim3(TPB), 0, s, (size_t)nc, cursor, 0);
  hipLaunchKernelGGL(k_count, dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, lv.agg, cnt);
  AMG_TRY(scan_excl(T, cnt, nc, lv.member_off, s));
  hipLaunchKernelGGL(k_scatter_members, dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, lv.agg, lv.member_off, cursor,
                     lv.members);
  hipLaunchKernelGGL(k_sort_members, dim3(nblk(nc)), dim3(TPB), 0, s, nc, lv.member_off, lv.members);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

// ------------------------------------------------------------------ layouts and their autotuner
struct SellLayout {
  int lc, lk, sort;  // log2 slice height, log2 lanes per row, rows sorted inside 64-row groups
};

// Device arrays of one sliced-ELL layout of a level.
struct SellArrays {
  int nslices = 0;
  int64_t entries = 0;
  int* w = nullptr;
  int* off = nullptr;
  int* perm = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  float* valf = nullptr;
};

// Row order and slice widths of a layout, and its entry count (padding
// included).  `alloc(void**, bytes)` provides the arrays that are kept.
template <typename Alloc>
int32_t layout_shape(Temps& T, const Level& lv, SellLayout L, Alloc&& alloc, SellArrays* A, hipStream_t s) {
  const int C = 1 << L.lc;
  A->nslices = (lv.n + C - 1) / C;
  const int nslots = A->nslices * C;
  if (L.sort) {
    AMG_TRY(alloc((void**)&A->perm, sizeof(int) * (size_t)lv.n + 16));
    hipLaunchKernelGGL(k_sell_perm, dim3(nblk(lv.n)), dim3(256), 0, s, lv.n, lv.row_ptr, A->perm);
  }
  AMG_TRY(alloc((void**)&A->w, sizeof(int) * (size_t)A->nslices + 16));
  AMG_TRY(alloc((void**)&A->off, sizeof(int) * ((size_t)A->nslices + 1) + 16));
  int* len = nullptr;
  AMG_TRY(T.get(&len, A->nslices));
  hipLaunchKernelGGL(k_sell_width, dim3(nblk(nslots)), dim3(TPB), 0, s, nslots, lv.n, lv.row_ptr, A->perm, L.lc,
                     L.lk, A->w);
  hipLaunchKernelGGL(k_sell_len, dim3(nblk(A->nslices)), dim3(TPB), 0, s, A->nslices, A->w, L.lc + L.lk, len);
  AMG_HIP(hipGetLastError());
  // total entries in int64 to guard against overflow of the int32 offsets
  std::vector<int> wh(A->nslices);
  AMG_HIP(hipMemcpyAsync(wh.data(), A->w, sizeof(int) * A->nslices, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  int64_t total = 0;
  for (int x : wh) total += (int64_t)x << (L.lc + L.lk);
  if (total >= (int64_t)1 << 31) {
    set_last_error("level too large for 32-bit sliced-ELL offsets");
    return AMG_ERR_ARG;
  }
  A->entries = total;
  AMG_TRY(scan_excl(T, len, A->nslices, A->off, s));
  AMG_HIP(hipStreamSynchronize(s));
  T.release(len);
  return AMG_OK;
}

// Column indices and weights of a layout whose shape is known.
template <typename Alloc>
int32_t layout_fill(const Level& lv, SellLayout L, bool f64, bool f32, Alloc&& alloc, SellArrays* A, hipStream_t s) {
  const size_t e = (size_t)std::max<int64_t>(A->entries, 1);
  AMG_TRY(alloc((void**)&A->col, sizeof(int) * e + 16));
  if (f64) AMG_TRY(alloc((void**)&A->val, sizeof(double) * e + 16));
  if (f32) AMG_TRY(alloc((void**)&A->valf, sizeof(float) * e + 16));
  const int nslots = A->nslices << L.lc;
  hipLaunchKernelGGL(k_sell_fill, dim3(nblk(nslots)), dim3(TPB), 0, s, nslots, lv.n, lv.row_ptr, lv.col, lv.W,
                     A->perm, L.lc, L.lk, A->off, A->w, A->col, A->val, A->valf);
  AMG_HIP(hipGetLastError());
  return AMG_OK;
}

void install(Level& lv, SellLayout L, const SellArrays& A) {
  lv.nslices = A.nslices;
  lv.sell_entries = A.entries;
  lv.sell_lc = L.lc;
  lv.sell_lk = L.lk;
  lv.sell_perm = A.perm;
  lv.sell_w = A.w;
  lv.sell_off = A.off;
  lv.sell_col = A.col;
  lv.sell_val = A.val;
  lv.sell_valf = A.valf;
}

// Candidate layouts: slice heights 64/32/16/8 with one lane per row, 32 rows
// x 2 lanes, 16 rows x 4 lanes; each unsorted and sorted.  The first is the
// plain layout (one wavefront per slice, rows in order).
constexpr SellLayout kLayouts[] = {{6, 0, 0}, {5, 0, 0}, {4, 0, 0}, {3, 0, 0}, {6, 0, 1}, {5, 0, 1}, {4, 0, 1},
                                   {3, 0, 1}, {5, 1, 0}, {5, 1, 1}, {4, 2, 0}, {4, 2, 1}};
constexpr int kNumLayouts = sizeof(kLayouts) / sizeof(kLayouts[0]);
// Levels with at least this many rows are tuned by timing; on smaller ones a
// launch takes a few microseconds, mostly latency, and the byte model decides.
constexpr int kTuneMinRows = 1 << 18;
// A sorted layout reads the row order and stages its reductions: the model
// takes it only when it saves more than this fraction of the bytes.
constexpr double kSortedPenalty = 1.10;
// The timed best replaces the model's choice only when faster by this factor.
constexpr double kTimedMargin = 0.97;

int ilog2(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

// Chooses the layout of a level.  Model: bytes of one pass over the layout
// (column index and weight per stored entry, plus the row order when
// sorted), the fewest winning.  Tuning (large levels): the storing Chebyshev
// step -- the solve's dominant kernel -- timed on each candidate whose model
// is within 1.5x of the best; the fastest replaces the model's choice if it
// is clearly faster.  Every layout gives the same results bit for bit (the row
// sums and the reductions have a fixed order), so the choice only affects
// speed.
int32_t choose_layout(amg_hier* h, Temps& T, Level& lv, bool mixed, hipStream_t s, SellLayout* best) {
  const amg_params& p = h->p;
  if (!p.autotune) {
    *best = SellLayout{ilog2(p.slice_height), ilog2(p.lanes_per_row), p.sort_rows ? 1 : 0};
    return AMG_OK;
  }
  auto tmp = [&](void** q, size_t bytes) -> int32_t {
    char* c = nullptr;
    AMG_TRY(T.get(&c, bytes));
    *q = c;
    return AMG_OK;
  };
  const double mt = mixed ? 4.0 : 8.0;
  double model[kNumLayouts];
  double best_model = 0.0;
  for (int c = 0; c < kNumLayouts; ++c) {
    SellArrays A;
    AMG_TRY(layout_shape(T, lv, kLayouts[c], tmp, &A, s));
    model[c] = ((double)A.entries * (4.0 + mt) + (kLayouts[c].sort ? 4.0 * lv.n : 0.0)) *
               (kLayouts[c].sort ? kSortedPenalty : 1.0);
    if (c == 0 || model[c] < best_model) best_model = model[c];
    T.release(A.perm);
    T.release(A.w);
    T.release(A.off);
  }
  int mi = 0;
  for (int c = 1; c < kNumLayouts; ++c)
    if (model[c] < model[mi]) mi = c;
  if (lv.n < kTuneMinRows) {
    *best = kLayouts[mi];
    return AMG_OK;
  }
  const size_t vt = mixed ? sizeof(float) : sizeof(double);
  char *wk = nullptr, *wb = nullptr, *y = nullptr;
  AMG_TRY(T.get(&wk, vt * lv.n));
  AMG_TRY(T.get(&wb, vt * lv.n));
  AMG_TRY(T.get(&y, vt * lv.n));
  AMG_HIP(hipMemsetAsync(wk, 0, vt * lv.n, s));
  AMG_HIP(hipMemsetAsync(wb, 0, vt * lv.n, s));
  AMG_HIP(hipMemsetAsync(y, 0, vt * lv.n, s));
  int bi = mi;
  float best_ms = 0.f, model_ms = 0.f;
  for (int c = 0; c < kNumLayouts; ++c) {
    if (c != mi && model[c] > 1.5 * best_model) continue;
    SellArrays A;
    AMG_TRY(layout_shape(T, lv, kLayouts[c], tmp, &A, s));
    AMG_TRY(layout_fill(lv, kLayouts[c], !mixed, mixed, tmp, &A, s));
    Level cand = lv;
    install(cand, kLayouts[c], A);
    float ms = 0.f;
    AMG_TRY(time_cheb_layout(cand, mixed, wk, wb, y, s, &ms));
    if (c == mi) model_ms = ms;
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      bi = c;
    }
    for (void* q : {(void*)A.perm, (void*)A.w, (void*)A.off, (void*)A.col, (void*)A.val, (void*)A.valf}) T.release(q);
  }
  T.release(wk);
  T.release(wb);
  T.release(y);
  *best = (best_ms < kTimedMargin * model_ms) ? kLayouts[bi] : kLayouts[mi];
  return AMG_OK;
}

int32_t build_sell(amg_hier* h, Temps& T, Level& lv, bool mixed, hipStream_t s) {
  if (mixed) {
    AMG_TRY(dalloc(h, &lv.Df, lv.n));
    hipLaunchKernelGGL(k_to_float, dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, lv.D, lv.Df);
    AMG_HIP(hipGetLastError());
  }
  SellLayout L;
  AMG_TRY(choose_layout(h, T, lv, mixed, s, &L));
  auto keep = [&](void** q, size_t bytes) -> int32_t { return dalloc(h, q, bytes); };
  SellArrays A;
  AMG_TRY(layout_shape(T, lv, L, keep, &A, s));
  AMG_TRY(layout_fill(lv, L, true, mixed, keep, &A, s));
  install(lv, L, A);
  // the tail program's plain layout of small levels
  if (lv.n <= kTailMaxRows) {
    const SellLayout P{6, 0, 0};
    SellArrays B = A;
    if (L.lc != P.lc || L.lk != P.lk || L.sort != P.sort) {
      B = SellArrays{};
      AMG_TRY(layout_shape(T, lv, P, keep, &B, s));
      AMG_TRY(layout_fill(lv, P, true, mixed, keep, &B, s));
    }
    lv.plain_nslices = B.nslices;
    lv.plain_entries = B.entries;
    lv.plain_off = B.off;
    lv.plain_w = B.w;
    lv.plain_col = B.col;
    lv.plain_val = B.val;
    lv.plain_valf = B.valf;
  }
  return AMG_OK;
}

// Chebyshev coefficients of eta * q_m in t = (x - theta)/eta (best uniform
// approximation to 1/x on [lambda1/ratio, lambda1]); stored divided by eta.
void smoother_coefficients(Level& lv, int m, double ratio) {
  const double l1 = lv.lambda1, l0 = l1 / ratio;
  lv.theta = 0.5 * (l1 + l0);
  lv.eta = 0.5 * (l1 - l0);
  const double kappa = l1 / l0;
  const double sk = std::sqrt(kappa);
  const double dl = (sk - 1.0) / (sk + 1.0);
  const double om = 1.0 - dl * dl;
  std::vector<double> c(m + 1, 0.0);
  if (m == 0) {
    c[0] = 2.0 * dl * (1.0 + dl * dl) / (om * om);
  } else {
    c[0] = 2.0 * dl / om;
    double pw = 1.0;
    for (int k = 1; k <= m; ++k) {
      pw *= -dl;
      c[k] = (k < m) ? 4.0 * dl * pw / om : 4.0 * dl * pw / (om * om);
    }
  }
  lv.coef.resize(m + 1);
  for (int k = 0; k <= m; ++k) lv.coef[k] = c[k] / lv.eta;
}

}  // namespace

int32_t build_hierarchy(amg_hier* h, int32_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                        const double* d, hipStream_t s) {
  const amg_params& p = h->p;
  auto t_setup = clk::now();
  double t_agg = 0.0, t_gal = 0.0;
  int total_rounds = 0;
  Temps T;
  bool pure_neumann = true;  // coarse d are sums of fine d (all >= 0)
  for (int32_t i = 0; i < n && pure_neumann; ++i) pure_neumann = d[i] == 0.0;

  Level l0;
  l0.n = n;
  l0.nnz = row_ptr[n];
  AMG_TRY(dalloc(h, &l0.row_ptr, n + 1));
  AMG_TRY(dalloc(h, &l0.col, std::max<int64_t>(l0.nnz, 1)));
  AMG_TRY(dalloc(h, &l0.W, std::max<int64_t>(l0.nnz, 1)));
  AMG_TRY(dalloc(h, &l0.d, n));
  AMG_TRY(dalloc(h, &l0.D, n));
  AMG_HIP(hipMemcpyAsync(l0.row_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, s));
  if (l0.nnz > 0) {
    AMG_HIP(hipMemcpyAsync(l0.col, col, sizeof(int32_t) * l0.nnz, hipMemcpyHostToDevice, s));
    AMG_HIP(hipMemcpyAsync(l0.W, w, sizeof(double) * l0.nnz, hipMemcpyHostToDevice, s));
  }
  AMG_HIP(hipMemcpyAsync(l0.d, d, sizeof(double) * n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_row_sums, dim3(nblk(n)), dim3(TPB), 0, s, n, l0.row_ptr, l0.W, l0.d, l0.D);
  AMG_HIP(hipGetLastError());
  h->lv.clear();
  h->lv.push_back(l0);

  const int passes = std::max(1, (int)std::lround(std::log2((double)p.agg_size)));
  const int raw = p.match_key == AMG_KEY_RAW;
  while (h->lv.back().n > p.coarse_max && (int)h->lv.size() < AMG_MAX_LEVELS) {
    Level& cur = h->lv.back();
    Graph g{cur.n, (int)cur.nnz, cur.row_ptr, cur.col, cur.W, cur.d, cur.D};
    int* agg = nullptr;
    Temps TL;  // intermediate pass graphs of this level
    if (p.aggregation == AMG_AGG_MIS) {
      Graph c;
      int rounds = 0;
      AMG_TRY(mis_level(h, TL, g, p.mis_distance, &agg, &c, &rounds, &t_agg, &t_gal, s));
      total_rounds += rounds;
      g = c;
    } else {
      AMG_TRY(dalloc(h, &agg, cur.n));
      hipLaunchKernelGGL(k_iota, dim3(nblk(cur.n)), dim3(TPB), 0, s, cur.n, agg);
    }
    for (int ps = 0; p.aggregation != AMG_AGG_MIS && ps < passes; ++ps) {
      auto ta = clk::now();
      int* mate = nullptr;
      AMG_TRY(TL.get(&mate, g.n));
      int rounds = 0;
      AMG_TRY(match_pass(TL, g, raw, p.tie_break == AMG_TIE_HASH, mate, &rounds, s));
      total_rounds += rounds;
      t_agg += ms_since(ta);
      Graph c;
      int* ids = nullptr;
      AMG_TRY(galerkin_pass(h, TL, g, mate, ps == passes - 1, &c, &ids, &t_agg, &t_gal, s));
      hipLaunchKernelGGL(k_compose, dim3(nblk(cur.n)), dim3(TPB), 0, s, cur.n, agg, ids);
      AMG_HIP(hipGetLastError());
      g = c;
    }
    AMG_HIP(hipStreamSynchronize(s));
    if (g.n > p.stagnation * cur.n) break;  // stagnation: cur becomes the coarsest level
    cur.agg = agg;
    Level nl;
    nl.n = g.n;
    nl.nnz = g.nnz;
    nl.row_ptr = g.rp;
    nl.col = g.col;
    nl.W = g.W;
    nl.d = g.d;
    nl.D = g.D;
    AMG_TRY(build_members(h, T, cur, g.n, s));
    h->lv.push_back(nl);
  }
  h->L = (int)h->lv.size() - 1;
  Level& co = h->lv.back();
  if (co.n > p.max_coarsest) {
    set_last_error("coarsening stagnated at " + std::to_string(co.n) + " rows");
    return AMG_ERR_COARSEN;
  }
  // lambda1 and the smoother of every level but the coarsest
  unsigned long long* lmax = nullptr;
  AMG_TRY(T.get(&lmax, AMG_MAX_LEVELS));
  hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, (size_t)AMG_MAX_LEVELS, lmax, 0ull);
  for (int l = 0; l <= h->L; ++l) {
    Level& lv = h->lv[l];
    hipLaunchKernelGGL(k_rowabs_max, dim3(nblk(lv.n)), dim3(TPB), 0, s, lv.n, lv.row_ptr, lv.W, lv.D, lmax + l);
  }
  AMG_HIP(hipGetLastError());
  std::vector<unsigned long long> lh(AMG_MAX_LEVELS);
  AMG_HIP(hipMemcpyAsync(lh.data(), lmax, sizeof(unsigned long long) * AMG_MAX_LEVELS, hipMemcpyDeviceToHost, s));
  AMG_HIP(hipStreamSynchronize(s));
  for (int l = 0; l <= h->L; ++l) {
    double v;
    std::memcpy(&v, &lh[l], sizeof(double));
    h->lv[l].lambda1 = v;
    if (l < h->L) smoother_coefficients(h->lv[l], p.degree, p.lambda0_ratio);
  }
  // coarsest: dense matrix and its Cholesky factor
  h->nL = co.n;
  AMG_TRY(dalloc(h, &h->chol, (size_t)co.n * co.n));
  hipLaunchKernelGGL(k_fill<double>, dim3(nblk((int64_t)co.n * co.n)), dim3(TPB), 0, s, (size_t)co.n * co.n,
                     h->chol, 0.0);
  hipLaunchKernelGGL(k_dense, dim3(nblk(co.n)), dim3(TPB), 0, s, co.n, co.row_ptr, co.col, co.W, co.D, h->chol);
  if (pure_neumann) {
    // d = 0 everywhere: A_L is singular with the constants as kernel (connected
    // graph); A_L + (1/n_L) 1 1^T is SPD and acts as a pseudo-inverse on
    // right-hand sides orthogonal to 1
    hipLaunchKernelGGL(k_add_const, dim3(nblk((int64_t)co.n * co.n)), dim3(TPB), 0, s, (size_t)co.n * co.n,
                       h->chol, 1.0 / co.n);
  }
  int* st = nullptr;
  AMG_TRY(T.get(&st, 1));
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(1024), 0, s, co.n, h->chol, st);
  AMG_HIP(hipGetLastError());
  int bad = 0;
  AMG_TRY(read_int(st, &bad, s));
  if (bad) {
    set_last_error("coarsest matrix is not positive definite");
    return AMG_ERR_SINGULAR;
  }
  if (co.n <= 1024) {
    AMG_TRY(dalloc(h, &h->chol_inv, (size_t)co.n * co.n));
    AMG_TRY(dalloc(h, &h->chol_invT, (size_t)co.n * co.n));
    hipLaunchKernelGGL(k_tri_inv, dim3(1), dim3(1024), 0, s, co.n, h->chol, h->chol_inv, h->chol_invT);
    AMG_HIP(hipGetLastError());
  }
  // solve-phase layouts: every level that is smoothed, and always the finest
  // level (outer-iteration products and residuals), even when it is the coarsest
  auto t_tune = clk::now();
  for (int l = 0; l < std::max(h->L, 1); ++l) AMG_TRY(build_sell(h, T, h->lv[l], h->mixed, s));
  AMG_HIP(hipStreamSynchronize(s));
  const double layout_ms = ms_since(t_tune);

  amg_hier_desc& ds = h->desc;
  std::memset(&ds, 0, sizeof(ds));
  ds.levels = (int)h->lv.size();
  ds.degree = h->p.degree;
  double gsum = 0.0, osum = 0.0;
  for (int l = 0; l <= h->L; ++l) {
    ds.n[l] = h->lv[l].n;
    ds.nnz[l] = h->lv[l].nnz;
    ds.lambda1[l] = h->lv[l].lambda1;
    gsum += h->lv[l].n;
    osum += (double)h->lv[l].nnz + h->lv[l].n;
  }
  ds.grid_complexity = gsum / h->lv[0].n;
  ds.operator_complexity = osum / ((double)h->lv[0].nnz + h->lv[0].n);
  ds.aggregation_ms = t_agg;
  ds.galerkin_ms = t_gal;
  ds.match_rounds = total_rounds;
  ds.precision = p.precision;
  ds.layout_ms = layout_ms;
  for (int l = 0; l < std::max(h->L, 1); ++l) {
    const Level& lv = h->lv[l];
    ds.slice_height[l] = 1 << lv.sell_lc;
    ds.lanes_per_row[l] = 1 << lv.sell_lk;
    ds.sorted_rows[l] = lv.sell_perm ? 1 : 0;
    ds.sell_entries[l] = lv.sell_entries;
  }
  ds.setup_ms = ms_since(t_setup);
  return AMG_OK;
}

}  // namespace amg
