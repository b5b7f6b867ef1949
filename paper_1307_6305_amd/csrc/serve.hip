// Serving with continuous batching: an incremental server (create, submit
// requests as they come, poll completions, destroy) and, built on it, the
// replay of an open-loop request stream.
//
// A server thread runs the loop below over the requests submitted so far, in
// submission order.  A request names a graph (by the caller's
// id; its data is set up once and the hierarchy stays resident) and carries
// one or more right-hand sides.  The batched mode keeps a set of in-flight
// right-hand sides ("slots"): between rounds of outer iterations it admits
// newly arrived right-hand sides as slots and device memory free up, and
// retires the converged ones; every round advances all in-flight slots
// together through the batched executor, so work of requests on different
// graphs overlaps on the device.  Hierarchies of new graphs are built by a
// setup thread on its own stream while the solves run.  Admission is against a
// device-memory budget (hierarchies, slot workspaces, schedules); idle
// hierarchies are evicted least recently used first.  The sequential mode
// solves one right-hand side at a time in arrival order with amg_solve, for
// comparison.  Each slot's arithmetic is independent of the other slots, so a
// result is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"
#include "hier.h"

namespace amg {
namespace {

using clk = std::chrono::steady_clock;

__global__ void k_zero_count(int* c) { *c = 0; }

// u = 0 (a fill kernel rather than a memset node)
__global__ void k_zero_vec(double* u, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[i] = 0.0;
}

struct Resident {
  amg_hier* h = nullptr;
  size_t bytes = 0;
  int in_flight = 0;  // slots using it
  double last_use = 0.0;
  std::vector<amg_hier*> spare;  // workspace clones kept for reuse
  size_t clone_bytes = 0;
  bool own_lent = false;         // the hierarchy's own workspace serves a slot
  bool failed = false;
  int32_t status = AMG_OK;
};

struct Req;

struct Slot {
  Req* rq = nullptr;
  int rhs = -1;
  Resident* res = nullptr;
  amg_hier* ws = nullptr;  // hierarchy or clone whose workspace it uses
  bool own_ws = false;     // ws is the resident hierarchy itself
  double* f = nullptr;
  double* u = nullptr;
  ItemState* st = nullptr;
  double admit_s = 0.0;
};

size_t hier_bytes(const amg_hier* h) { return h->bytes; }

// Device vectors of the slots (right-hand side and solution), kept in size
// classes (powers of two, at least 4096 doubles) and reused, so that admitting
// and retiring right-hand sides allocates nothing once the pool holds enough
// buffers (a free would also synchronize the whole device).
struct VecPool {
  std::map<size_t, std::vector<double*>> idle;  // class (doubles) -> idle buffers
  size_t held = 0;                               // device bytes of every buffer
  static size_t cls(size_t n) {
    size_t c = 4096;
    while (c < n) c <<= 1;
    return c;
  }
  // bytes a get(n) would have to allocate
  size_t need(size_t n) const {
    auto it = idle.find(cls(n));
    return it != idle.end() && !it->second.empty() ? 0 : cls(n) * sizeof(double);
  }
  int32_t get(size_t n, double** out) {
    auto& v = idle[cls(n)];
    if (!v.empty()) {
      *out = v.back();
      v.pop_back();
      return AMG_OK;
    }
    AMG_HIP(hipMalloc(out, cls(n) * sizeof(double)));
    held += cls(n) * sizeof(double);
    return AMG_OK;
  }
  void put(double* p, size_t n) { idle[cls(n)].push_back(p); }
  // frees the idle buffers (under memory pressure); returns the bytes freed
  size_t release_idle() {
    size_t b = 0;
    for (auto& kv : idle) {
      for (double* p : kv.second) (void)hipFree(p);
      b += kv.first * sizeof(double) * kv.second.size();
      kv.second.clear();
    }
    held -= b;
    return b;
  }
};

// One submitted request: the caller's record, with the right-hand sides and
// (when given) the graph copied in; u stays the caller's.
struct Req {
  amg_request q;
  int ticket = 0;
  int remaining = 0;  // right-hand sides not yet completed
  std::vector<double> f;
  std::vector<int32_t> rp, col;
  std::vector<double> w, d;
};

// Fraction of the memory budget that releases bring the server down to.
constexpr double kLowWater = 0.9;

struct Server {
  amg_serve_cfg cfg;
  hipStream_t s = nullptr;       // solve stream
  hipStream_t s_setup = nullptr; // setup stream
  int device = 0;
  clk::time_point t0;
  size_t bytes = 0, peak = 0;
  int evictions = 0, setups = 0, steps = 0, max_in_flight = 0;
  // where the serve loop's time goes (seconds)
  double t_schedule = 0.0, t_admit = 0.0, t_release = 0.0, t_iterate = 0.0;

  std::map<int, Resident*> resident;
  VecPool pool;                     // slot vectors (serve loop thread only)
  std::mutex mu;                    // guards the request list, outbox, `resident` setup fields, setup queue
  std::condition_variable cv;       // new request, setup done, closing
  std::condition_variable cv_out;   // new completions
  std::deque<std::unique_ptr<Req>> reqs;  // submitted requests (elements never move)
  bool closing = false;             // no more submissions: finish and stop
  std::deque<amg_completion> outbox;
  int outstanding = 0;              // right-hand sides submitted and not yet completed
  std::deque<Req*> setup_queue;     // requests whose graph needs a setup
  std::map<int, size_t> setup_pending;  // graph id -> bytes reserved while queued or running
  bool stop_worker = false;
  std::thread loop_thread;
  int32_t loop_status = AMG_OK;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

  void note_bytes() { peak = std::max(peak, bytes); }

  // ---------------------------------------------------------------- setup thread
  void worker() {
    (void)hipSetDevice(device);
    for (;;) {
      Req* rq;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop_worker || !setup_queue.empty(); });
        if (stop_worker && setup_queue.empty()) return;
        rq = setup_queue.front();
        setup_queue.pop_front();
      }
      const amg_request& q = rq->q;
      amg_hier* h = nullptr;
      const int32_t st = amg_setup(q.n, q.row_ptr, q.col, q.w, q.d, &cfg.params, s_setup, &h);
      std::lock_guard<std::mutex> lk(mu);
      Resident* R = new Resident();
      R->h = h;
      R->status = st;
      R->failed = st != AMG_OK;
      R->bytes = h ? hier_bytes(h) : 0;
      R->last_use = now();
      resident[q.graph_id] = R;
      // the reservation made when the setup was queued becomes the actual size
      bytes -= setup_pending[q.graph_id];
      setup_pending.erase(q.graph_id);
      ++setups;
      bytes += R->bytes;
      note_bytes();
      cv.notify_all();
    }
  }

  // ---------------------------------------------------------------- memory
  // Upper bound of a hierarchy's device bytes from the graph size: level data
  // (CSR, sliced ELL, FP32 copies, aggregation maps) over all levels and the
  // solve workspace, with room for coarse levels and padding.
  size_t setup_estimate(const amg_request& q) const {
    const size_t n = (size_t)q.n, nnz = (size_t)q.row_ptr[q.n];
    const bool mixed = cfg.params.precision == AMG_MIXED;
    const size_t vt = mixed ? 4 : 8;
    // sliced-ELL entries of the plain layout (64-row slices, rows in order);
    // the layout the autotuner keeps stores at most 1.5x that many
    size_t e64 = 0;
    for (size_t s0 = 0; s0 < n; s0 += 64) {
      int w = 0;
      for (size_t r = s0; r < std::min(n, s0 + 64); ++r) w = std::max(w, q.row_ptr[r + 1] - q.row_ptr[r]);
      e64 += 64 * (size_t)w;
    }
    const size_t sell = (3 * e64) / 2 + 64;
    // finest level: CSR + d, D; sliced ELL (+ row order); FP32 copies; aggregation maps
    size_t level0 = 4 * (n + 1) + 12 * nnz + 16 * n + 12 * sell + 4 * n + 12 * n;
    if (mixed) level0 += 4 * sell + 4 * n;
    // coarser levels shrink at least twofold per level: at most as much again
    const size_t data = 2 * level0;
    // outer FCG vectors, the finest level's cycle vectors, coarse-level vectors
    const size_t work = (16 + 16 * (size_t)cfg.params.restart + 4 * vt) * n +
                        (7 + 2 * (size_t)cfg.params.inner_steps) * vt * n;
    return data + work + (64 << 10);
  }

  int resident_busy() const {
    int b = 0;
    for (const auto& kv : resident) b += kv.second->in_flight;
    return b;
  }

  // Evict idle hierarchies (least recently used first) until `need` more
  // bytes fit the budget; `keep` (the hierarchy the room is for) is never
  // evicted.  Caller holds mu.
  bool make_room(size_t need, const Resident* keep = nullptr) {
    auto over = [&] { return (double)(bytes + need) > cfg.hbm_budget_bytes; };
    if (!over()) return true;
    // Once the budget binds, release down to a low-water mark (90 % of the
    // budget) rather than just enough: every release waits for the device to
    // drain (hipFree), so releasing in bulk pays that wait once for many
    // admissions instead of once per admission.
    auto over_low = [&] { return (double)(bytes + need) > kLowWater * cfg.hbm_budget_bytes; };
    const auto tr0 = clk::now();
    struct Tally {  // adds the time spent here to t_release however it returns
      double& t;
      clk::time_point t0;
      ~Tally() { t += std::chrono::duration<double>(clk::now() - t0).count(); }
    } tally{t_release, tr0};
    bytes -= pool.release_idle();
    // then idle workspace clones, those of the least recently used hierarchy
    // first (a clone is rebuilt in milliseconds, a hierarchy needs a setup)
    while (over_low()) {
      Resident* from = nullptr;
      for (auto& kv : resident) {
        Resident* R = kv.second;
        if (R != keep && !R->spare.empty() && (!from || R->last_use < from->last_use)) from = R;
      }
      if (!from) break;
      amg_hier* c = from->spare.back();
      from->spare.pop_back();
      const size_t b = c->bytes;
      free_clone(c);
      from->clone_bytes -= b;
      bytes -= b;
    }
    while (over()) {
      Resident* victim = nullptr;
      int vid = 0;
      for (auto& kv : resident) {
        Resident* R = kv.second;
        if (R != keep && R->in_flight == 0 && !R->failed && (!victim || R->last_use < victim->last_use)) {
          victim = R;
          vid = kv.first;
        }
      }
      if (!victim) return false;
      for (amg_hier* c : victim->spare) free_clone(c);
      bytes -= victim->bytes + victim->clone_bytes;
      amg_free(victim->h);
      delete victim;
      resident.erase(vid);
      ++evictions;
    }
    return true;
  }

  // One more right-hand side of rq is finished; after the last one the
  // request's copies of its right-hand sides and graph go (a long stream
  // would otherwise hold every request's data until the server ends).  The
  // graph copy stays while a setup of that graph is queued or running (the
  // setup thread may be reading it).  Caller holds mu.
  void rhs_done(Req* rq) {
    if (--rq->remaining > 0) return;
    std::vector<double>().swap(rq->f);
    rq->q.f = nullptr;
    if (!setup_pending.count(rq->q.graph_id)) {
      std::vector<int32_t>().swap(rq->rp);
      std::vector<int32_t>().swap(rq->col);
      std::vector<double>().swap(rq->w);
      std::vector<double>().swap(rq->d);
      rq->q.row_ptr = rq->q.col = nullptr;
      rq->q.w = rq->q.d = nullptr;
    }
  }

  // Records a finished right-hand side in the outbox.  Caller holds mu.
  void complete(const Slot& sl, int32_t status, int iters, double rel_true) {
    amg_completion c;
    c.request = sl.rq->ticket;
    c.rhs = sl.rhs;
    c.status = status;
    c.iters = iters;
    c.rel_res_true = rel_true;
    c.arrival_s = sl.rq->q.arrival_s;
    c.admit_s = sl.admit_s;
    c.finish_s = now();
    outbox.push_back(c);
    --outstanding;
    rhs_done(sl.rq);
    cv_out.notify_all();
  }

  // Caller holds mu.
  void fail_request(Req* rq, int32_t status, int first_rhs = 0) {
    const double t = now();
    for (int k = first_rhs; k < rq->q.nrhs; ++k) {
      amg_completion c;
      c.request = rq->ticket;
      c.rhs = k;
      c.status = status;
      c.iters = 0;
      c.rel_res_true = 0.0;
      c.arrival_s = rq->q.arrival_s;
      c.admit_s = t;
      c.finish_s = t;
      outbox.push_back(c);
      --outstanding;
      rhs_done(rq);
    }
    cv_out.notify_all();
  }

  // The request at position i of the submission order, or null if not (yet)
  // submitted; `done` tells whether nothing more will come.
  Req* request_at(size_t i, bool* done) {
    std::lock_guard<std::mutex> lk(mu);
    *done = closing && i >= reqs.size();
    return i < reqs.size() ? reqs[i].get() : nullptr;
  }

  // ---------------------------------------------------------------- batched mode
  // A submitted request with right-hand sides not yet admitted.
  struct Pending {
    Req* rq;
    int next_rhs;
  };

  int32_t run_batched() {
    std::thread th([this] { worker(); });
    struct Joiner {
      Server* S;
      std::thread* t;
      ~Joiner() {
        {
          std::lock_guard<std::mutex> lk(S->mu);
          S->stop_worker = true;
        }
        S->cv.notify_all();
        t->join();
      }
    } joiner{this, &th};

    size_t scanned = 0;              // requests moved from the submission list to `pending`
    std::vector<Pending> pending;    // in submission order
    std::vector<Slot> active;        // in the iteration schedule, iterating
    std::vector<Slot> fresh;         // admitted in this round, not yet started
    ItemState* d_states = nullptr;   // pool of item states, one per slot position
    int* d_nactive = nullptr;
    const int max_slots = std::max(1, cfg.max_slots);
    std::vector<int> free_state(max_slots);
    for (int i = 0; i < max_slots; ++i) free_state[i] = max_slots - 1 - i;
    std::map<const void*, int> state_index;
    Schedule sched_iter, sched_aux;
    bool membership_changed = true;
    size_t sched_items = 0;          // items in sched_iter (active ones and retired ones)
    int32_t result = AMG_OK;

    auto cleanup = [&]() {
      (void)hipStreamSynchronize(s);
      schedule_free(&sched_iter);
      schedule_free(&sched_aux);
      for (std::vector<Slot>* v : {&active, &fresh})
        for (Slot& sl : *v) {
          if (sl.f) pool.put(sl.f, (size_t)sl.rq->q.n);
          if (sl.u) pool.put(sl.u, (size_t)sl.rq->q.n);
        }
      {
        std::lock_guard<std::mutex> lk(mu);
        bytes -= pool.release_idle();
      }
      if (d_states) (void)hipFree(d_states);
      if (d_nactive) (void)hipFree(d_nactive);
    };

    // The admission and iteration loop; a device error ends it early.
    auto loop = [&]() -> int32_t {
      AMG_HIP(hipMalloc(&d_states, sizeof(ItemState) * max_slots));
      AMG_HIP(hipMalloc(&d_nactive, sizeof(int)));
      // built after the allocation: the kernels take the counter's address from it
      const BatchCtl ctl{cfg.params.tol, cfg.params.max_iter, 0, d_nactive};
      while (true) {
        const double t = now();
        bool no_more = false;
        {
          std::lock_guard<std::mutex> lk(mu);
          for (; scanned < reqs.size(); ++scanned) pending.push_back(Pending{reqs[scanned].get(), 0});
          no_more = closing;
        }
        // --- queue setups for pending requests whose graph is not resident,
        //     reserving a conservative size estimate against the budget.  Only
        //     the oldest pending request's setup may evict idle hierarchies;
        //     later ones start early only in free room (otherwise they could
        //     evict the hierarchy the oldest needs, and the two would evict
        //     each other).
        {
          std::lock_guard<std::mutex> lk(mu);
          for (size_t k = 0; k < pending.size(); ++k) {
            Req* rq = pending[k].rq;
            const amg_request& q = rq->q;
            if (resident.count(q.graph_id) || setup_pending.count(q.graph_id)) continue;
            if (!q.row_ptr) continue;  // no data to set up: fails at admission
            const size_t est = setup_estimate(q);
            if (k > 0) {
              if ((double)(bytes + est) > cfg.hbm_budget_bytes) break;
            } else if (!make_room(est)) {
              if (active.empty() && resident_busy() == 0 && setup_pending.empty()) {
                // larger than the whole budget: nothing can ever make room
                Resident* R = new Resident();
                R->failed = true;
                R->status = AMG_ERR_BUDGET;
                resident[q.graph_id] = R;
              }
              break;  // later graphs wait for room too
            }
            bytes += est;
            note_bytes();
            setup_pending[q.graph_id] = est;
            setup_queue.push_back(rq);
          }
        }
        cv.notify_all();
        // --- admit pending right-hand sides while slots and memory allow, in
        //     submission order among requests whose graph is resident; a
        //     request whose graph is still being set up does not hold back
        //     later requests on resident graphs
        fresh.clear();
        bool stop = false;
        const auto ta0 = clk::now();
        const double rel0 = t_release;
        for (size_t k = 0; k < pending.size() && !stop;) {
          Pending& pd = pending[k];
          Req* rq = pd.rq;
          const amg_request& q = rq->q;
          std::unique_lock<std::mutex> lk(mu);
          auto it = resident.find(q.graph_id);
          if (it == resident.end()) {
            if (!q.row_ptr && !setup_pending.count(q.graph_id)) {  // evicted and no data: fail
              fail_request(rq, AMG_ERR_ARG, pd.next_rhs);
              pending.erase(pending.begin() + k);
              continue;
            }
            ++k;  // setup still running: later requests may go first
            continue;
          }
          Resident* R = it->second;
          if (R->failed) {
            fail_request(rq, R->status, pd.next_rhs);
            pending.erase(pending.begin() + k);
            continue;
          }
          bool removed = false;
          while (pd.next_rhs < q.nrhs) {
            if ((int)(active.size() + fresh.size()) >= max_slots || free_state.empty()) {
              stop = true;
              break;
            }
            // one slot: workspace (spare clone, the hierarchy's own, or a new clone) + f, u
            const size_t n = (size_t)q.n;
            amg_hier* ws = nullptr;
            bool own = false;
            size_t extra = 2 * pool.need(n) + 64;
            if (!R->spare.empty()) {
              ws = R->spare.back();
            } else if (!R->own_lent) {
              own = true;  // the hierarchy's own workspace is free
            } else {
              extra += clone_bytes_of(R->h);  // what make_clone allocates
            }
            if (!make_room(extra, R)) {
              if (active.empty() && fresh.empty()) {  // nothing will ever free memory: give up on it
                fail_request(rq, AMG_ERR_BUDGET, pd.next_rhs);
                pending.erase(pending.begin() + k);
                removed = true;
              } else {
                stop = true;
              }
              break;
            }
            if (!R->spare.empty()) {
              R->spare.pop_back();
            } else if (!own) {
              const int32_t st = make_clone(R->h, &ws, s);
              if (st != AMG_OK) return st;
              R->clone_bytes += ws->bytes;
              bytes += ws->bytes;
            }
            if (own) {
              ws = R->h;
              R->own_lent = true;
            }
            Slot sl;
            sl.rq = rq;
            sl.rhs = pd.next_rhs;
            sl.res = R;
            sl.ws = ws;
            sl.own_ws = own;
            sl.admit_s = std::max(t, q.arrival_s);  // submitted after this round began
            R->in_flight++;
            R->last_use = t;
            const int si = free_state.back();
            free_state.pop_back();
            sl.st = d_states + si;
            state_index[sl.st] = si;
            // the slot is accounted for from here on (an error fails it with the rest)
            fresh.push_back(sl);
            ++pd.next_rhs;
            Slot& fs = fresh.back();
            const size_t before = pool.held;
            AMG_TRY(pool.get(n, &fs.f));
            AMG_TRY(pool.get(n, &fs.u));
            bytes += pool.held - before;
            note_bytes();
            // the copy-in without the lock (submissions and polls go on)
            lk.unlock();
            AMG_HIP(hipMemcpyAsync(fs.f, q.f + (size_t)sl.rhs * n, n * sizeof(double), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_zero_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fs.u, (int)n);
            AMG_HIP(hipGetLastError());
            lk.lock();
          }
          if (removed) continue;
          if (pd.next_rhs >= q.nrhs) {
            pending.erase(pending.begin() + k);
            continue;
          }
          ++k;
        }
        // (releases made for admissions are counted in t_release)
        t_admit += std::chrono::duration<double>(clk::now() - ta0).count() - (t_release - rel0);
        // --- start the new slots: r = f - A u, activation
        if (!fresh.empty()) {
          std::vector<BatchItem> items;
          for (const Slot& sl : fresh) items.push_back(BatchItem{sl.ws, sl.f, sl.u, sl.st});
          const auto tb0 = clk::now();
          AMG_TRY(schedule_build(&sched_aux, SCHED_INIT, items, s));
          t_schedule += std::chrono::duration<double>(clk::now() - tb0).count();
          hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, d_nactive);
          AMG_TRY(schedule_run(&sched_aux, ctl, s));
          for (const Slot& sl : fresh) active.push_back(sl);
          fresh.clear();
          membership_changed = true;
        }
        if (active.empty()) {
          if (pending.empty() && no_more) {
            std::lock_guard<std::mutex> lk(mu);
            if (scanned == reqs.size()) break;  // closing and everything done
            continue;
          }
          // wait for a submission, a setup or the close
          std::unique_lock<std::mutex> lk(mu);
          cv.wait_for(lk, std::chrono::milliseconds(2));
          continue;
        }
        // --- one round of outer iterations over every in-flight slot.  The
        //     iteration schedule is rebuilt when slots have joined; retired
        //     slots stay in it as frozen items (their blocks return at once)
        //     until the next rebuild, or until they outnumber the live ones.
        if (membership_changed || 2 * active.size() < sched_items) {
          std::vector<BatchItem> items;
          for (const Slot& sl : active) items.push_back(BatchItem{sl.ws, sl.f, sl.u, sl.st});
          const auto tb0 = clk::now();
          AMG_TRY(schedule_build(&sched_iter, SCHED_ITER, items, s));
          t_schedule += std::chrono::duration<double>(clk::now() - tb0).count();
          sched_items = active.size();
          membership_changed = false;
        }
        max_in_flight = std::max(max_in_flight, (int)active.size());
        const auto ti0 = clk::now();
        for (int k = 0; k < std::max(1, cfg.iters_per_step); ++k) AMG_TRY(schedule_run(&sched_iter, ctl, s));
        ++steps;
        // --- retire converged slots
        std::vector<ItemState> hst(active.size());
        for (size_t i = 0; i < active.size(); ++i)
          AMG_HIP(hipMemcpyAsync(&hst[i], active[i].st, sizeof(ItemState), hipMemcpyDeviceToHost, s));
        AMG_HIP(hipStreamSynchronize(s));
        t_iterate += std::chrono::duration<double>(clk::now() - ti0).count();
        std::vector<Slot> done, keep;
        for (size_t i = 0; i < active.size(); ++i) (hst[i].active ? keep : done).push_back(active[i]);
        if (!done.empty()) {
          std::vector<BatchItem> items;
          for (const Slot& sl : done) items.push_back(BatchItem{sl.ws, sl.f, sl.u, sl.st});
          const auto tb0 = clk::now();
          AMG_TRY(schedule_build(&sched_aux, SCHED_FINAL, items, s));
          t_schedule += std::chrono::duration<double>(clk::now() - tb0).count();
          AMG_TRY(schedule_run(&sched_aux, ctl, s));
          std::vector<ItemState> fst(done.size());
          for (size_t i = 0; i < done.size(); ++i)
            AMG_HIP(hipMemcpyAsync(&fst[i], done[i].st, sizeof(ItemState), hipMemcpyDeviceToHost, s));
          for (const Slot& sl : done) {
            const amg_request& q = sl.rq->q;
            if (q.u)
              AMG_HIP(hipMemcpyAsync(q.u + (size_t)sl.rhs * q.n, sl.u, sizeof(double) * q.n, hipMemcpyDeviceToHost,
                                     s));
          }
          AMG_HIP(hipStreamSynchronize(s));
          std::lock_guard<std::mutex> lk(mu);
          for (size_t i = 0; i < done.size(); ++i) {
            const Slot& sl = done[i];
            const double rho0 = std::sqrt(fst[i].rr0);
            complete(sl, fst[i].status, fst[i].iter, rho0 > 0 ? std::sqrt(fst[i].rrt) / rho0 : 0.0);
            // the slot's buffers, state and workspace go back for reuse: the
            // iteration schedule still lists the slot, frozen, and is rebuilt
            // before any of them serves a new slot (new slots always rebuild it)
            pool.put(sl.f, (size_t)sl.rq->q.n);
            pool.put(sl.u, (size_t)sl.rq->q.n);
            sl.res->in_flight--;
            sl.res->last_use = now();
            if (sl.own_ws) sl.res->own_lent = false;
            else sl.res->spare.push_back(sl.ws);
            free_state.push_back(state_index[sl.st]);
            state_index.erase(sl.st);
          }
          active.swap(keep);
        }
      }
      return AMG_OK;
    };
    result = loop();
    if (result != AMG_OK) {
      // complete every admitted slot and every right-hand side not yet
      // admitted with the error; no further submissions are taken
      std::lock_guard<std::mutex> lk(mu);
      closing = true;
      for (std::vector<Slot>* v : {&active, &fresh})
        for (const Slot& sl : *v) complete(sl, result, 0, 0.0);
      for (const Pending& pd : pending) fail_request(pd.rq, result, pd.next_rhs);
      for (size_t k = scanned; k < reqs.size(); ++k) fail_request(reqs[k].get(), result, 0);
    }
    cleanup();
    return result;
  }

  // ---------------------------------------------------------------- sequential mode
  int32_t run_sequential() {
    size_t next = 0;  // the request being served
    int cur_rhs = 0;  // its first right-hand side not yet completed
    auto loop = [&]() -> int32_t {
      for (;; ++next) {
        cur_rhs = 0;
        Req* rq = nullptr;
        for (;;) {  // the next submission, or the end
          bool no_more = false;
          rq = request_at(next, &no_more);
          if (rq || no_more) break;
          std::unique_lock<std::mutex> lk(mu);
          cv.wait_for(lk, std::chrono::milliseconds(2));
        }
        if (!rq) break;
        const amg_request& q = rq->q;
        Resident* R = nullptr;
        auto it = resident.find(q.graph_id);
        if (it != resident.end()) {
          R = it->second;
        } else if (q.row_ptr) {
          R = new Resident();
          R->status = amg_setup(q.n, q.row_ptr, q.col, q.w, q.d, &cfg.params, s, &R->h);
          R->failed = R->status != AMG_OK;
          R->bytes = R->h ? hier_bytes(R->h) : 0;
          ++setups;
          if (!R->failed && !make_room(R->bytes)) {
            amg_free(R->h);
            R->h = nullptr;
            R->failed = true;
            R->status = AMG_ERR_BUDGET;
          }
          if (!R->failed) bytes += R->bytes;
          note_bytes();
          resident[q.graph_id] = R;
        }
        if (!R || R->failed) {
          std::lock_guard<std::mutex> lk(mu);
          fail_request(rq, R ? R->status : AMG_ERR_ARG);
          continue;
        }
        R->last_use = now();
        const double admit = now();
        double* f = nullptr;
        double* u = nullptr;
        {
          std::lock_guard<std::mutex> lk(mu);
          const size_t before = pool.held;
          if (!make_room(2 * pool.need((size_t)q.n), R)) {
            fail_request(rq, AMG_ERR_BUDGET);
            continue;
          }
          AMG_TRY(pool.get((size_t)q.n, &f));
          const int32_t st = pool.get((size_t)q.n, &u);
          if (st != AMG_OK) {
            pool.put(f, (size_t)q.n);
            return st;
          }
          bytes += pool.held - before;
          note_bytes();
        }
        struct Give {  // the vectors go back to the pool however the request ends
          VecPool& p;
          double* f;
          double* u;
          size_t n;
          ~Give() {
            p.put(f, n);
            p.put(u, n);
          }
        } give{pool, f, u, (size_t)q.n};
        for (int k = 0; k < q.nrhs; ++k) {
          AMG_HIP(hipMemcpyAsync(f, q.f + (size_t)k * q.n, q.n * sizeof(double), hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(k_zero_vec, dim3((unsigned)((q.n + 255) / 256)), dim3(256), 0, s, u, (int)q.n);
          AMG_HIP(hipGetLastError());
          amg_info info{};
          const int32_t st = solve(R->h, f, u, s, &info);
          if (q.u) AMG_HIP(hipMemcpyAsync(q.u + (size_t)k * q.n, u, q.n * sizeof(double), hipMemcpyDeviceToHost, s));
          AMG_HIP(hipStreamSynchronize(s));
          Slot sl;
          sl.rq = rq;
          sl.rhs = k;
          sl.admit_s = admit;
          std::lock_guard<std::mutex> lk(mu);
          complete(sl, st == AMG_OK || st == AMG_ERR_MAXIT || st == AMG_ERR_BREAKDOWN ? info.status : st, info.iters,
                   info.rel_res_true);
          cur_rhs = k + 1;
          ++steps;
        }
      }
      return AMG_OK;
    };
    const int32_t result = loop();
    if (result != AMG_OK) {
      std::lock_guard<std::mutex> lk(mu);
      closing = true;
      for (size_t k = next; k < reqs.size(); ++k) fail_request(reqs[k].get(), result, k == next ? cur_rhs : 0);
    }
    (void)hipStreamSynchronize(s);
    {
      std::lock_guard<std::mutex> lk(mu);
      bytes -= pool.release_idle();
    }
    return result;
  }

  ~Server() {
    if (loop_thread.joinable()) (void)finish();
    for (auto& kv : resident) {
      Resident* R = kv.second;
      for (amg_hier* c : R->spare) free_clone(c);
      if (R->h) amg_free(R->h);
      delete R;
    }
    if (s_setup) (void)hipStreamDestroy(s_setup);
  }

  // ---------------------------------------------------------------- the server thread
  void run() {
    (void)hipSetDevice(device);
    const int32_t st = cfg.mode == AMG_SERVE_SEQUENTIAL ? run_sequential() : run_batched();
    // a device error stops the loop; pollers see it in poll's return value
    std::lock_guard<std::mutex> lk(mu);
    loop_status = st;
    if (st != AMG_OK) closing = true;
    cv_out.notify_all();
  }

  int32_t start(const amg_serve_cfg& c, hipStream_t stream) {
    cfg = c;
    s = stream;
    (void)hipGetDevice(&device);
    AMG_HIP(hipStreamCreateWithFlags(&s_setup, hipStreamNonBlocking));
    t0 = clk::now();
    loop_thread = std::thread([this] { run(); });
    return AMG_OK;
  }

  // Copies the request in and queues it; `arrival` < 0 stamps the current time.
  int32_t submit(const amg_request& in, double arrival, int32_t* ticket) {
    auto rq = std::make_unique<Req>();
    rq->q = in;
    const size_t n = (size_t)in.n;
    rq->f.assign(in.f, in.f + (size_t)in.nrhs * n);
    rq->q.f = rq->f.data();
    if (in.row_ptr) {
      const size_t nnz = (size_t)in.row_ptr[in.n];
      rq->rp.assign(in.row_ptr, in.row_ptr + n + 1);
      rq->col.assign(in.col, in.col + nnz);
      rq->w.assign(in.w, in.w + nnz);
      rq->d.assign(in.d, in.d + n);
      rq->q.row_ptr = rq->rp.data();
      rq->q.col = rq->col.data();
      rq->q.w = rq->w.data();
      rq->q.d = rq->d.data();
    }
    std::lock_guard<std::mutex> lk(mu);
    if (closing) {
      set_last_error("server is closing");
      return AMG_ERR_ARG;
    }
    rq->q.arrival_s = arrival < 0 ? now() : arrival;
    rq->ticket = (int32_t)reqs.size();
    rq->remaining = in.nrhs;
    if (ticket) *ticket = rq->ticket;
    outstanding += in.nrhs;
    reqs.push_back(std::move(rq));
    cv.notify_all();
    return AMG_OK;
  }

  int32_t poll(amg_completion* out, int32_t max, double wait_s, int32_t* count) {
    std::unique_lock<std::mutex> lk(mu);
    if (outbox.empty() && wait_s > 0) {
      cv_out.wait_for(lk, std::chrono::duration<double>(wait_s),
                      [&] { return !outbox.empty() || (closing && outstanding == 0) || loop_status != AMG_OK; });
    }
    int32_t k = 0;
    while (k < max && !outbox.empty()) {
      out[k++] = outbox.front();
      outbox.pop_front();
    }
    *count = k;
    return loop_status;
  }

  // No more submissions: finish every submitted request and stop the thread.
  int32_t finish() {
    {
      std::lock_guard<std::mutex> lk(mu);
      closing = true;
    }
    cv.notify_all();
    if (loop_thread.joinable()) loop_thread.join();
    return loop_status;
  }

  void stats(amg_serve_stats* st) {
    if (!st) return;
    st->wall_s = now();
    st->peak_bytes = (double)peak;
    st->evictions = evictions;
    st->setups = setups;
    st->steps = steps;
    st->max_in_flight = max_in_flight;
    st->schedule_s = t_schedule;
    st->admit_s = t_admit;
    st->release_s = t_release;
    st->iterate_s = t_iterate;
  }
};

}  // namespace

int32_t server_create(const amg_serve_cfg& cfg, hipStream_t s, void** out) {
  auto S = std::make_unique<Server>();
  AMG_TRY(S->start(cfg, s));
  *out = S.release();
  return AMG_OK;
}

int32_t server_submit(void* srv, const amg_request& q, int32_t* ticket) {
  return static_cast<Server*>(srv)->submit(q, -1.0, ticket);
}

int32_t server_poll(void* srv, amg_completion* out, int32_t max, double wait_s, int32_t* count) {
  return static_cast<Server*>(srv)->poll(out, max, wait_s, count);
}

int32_t server_destroy(void* srv, amg_serve_stats* stats) {
  Server* S = static_cast<Server*>(srv);
  const int32_t st = S->finish();
  S->stats(stats);
  delete S;
  return st;
}

// Replay of a request stream on the incremental server: requests are
// submitted in arrival order -- at their arrival times when realtime, all at
// once otherwise -- and their completions gathered request-major.
int32_t serve(const amg_serve_cfg& cfg, const amg_request* reqs, int32_t nreq, amg_completion* out,
              amg_serve_stats* stats, hipStream_t s) {
  std::vector<int> order(nreq), base(nreq);
  int total = 0;
  for (int i = 0; i < nreq; ++i) {
    order[i] = i;
    base[i] = total;
    total += reqs[i].nrhs;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  std::memset(out, 0, sizeof(amg_completion) * total);
  Server S;
  AMG_TRY(S.start(cfg, s));
  std::vector<int> of_ticket(nreq);
  int32_t st = AMG_OK;
  for (int k = 0; k < nreq && st == AMG_OK; ++k) {
    const amg_request& q = reqs[order[k]];
    if (cfg.realtime) {
      const double wait = q.arrival_s - S.now();
      if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
    }
    int32_t ticket = 0;
    st = S.submit(q, q.arrival_s, &ticket);
    of_ticket[ticket] = order[k];
  }
  const int32_t fst = S.finish();
  if (st == AMG_OK) st = fst;
  for (const amg_completion& c : S.outbox) {
    const int r = of_ticket[c.request];
    amg_completion cc = c;
    cc.request = r;
    out[base[r] + c.rhs] = cc;
  }
  S.stats(stats);
  return st;
}

}  // namespace amg
