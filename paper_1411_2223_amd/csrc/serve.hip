// serve.hip -- request loop with continuous batching for CG solves.
//
// A scheduler thread owns "runs": one batch of column slots per (gauge field,
// precision mode), with its workspace carved from the caller's arena (the HBM
// budget) and its own HIP stream.  Every run advances in blocks of
// poll_iters CG iterations (one hipGraph replay).  Between blocks, queued
// requests join a run when enough contiguous column slots are free, finished
// columns retire, and their slots go back to the pool; runs of different
// fields overlap on the device through their streams.  A column's arithmetic
// depends only on its own data (per-column scalars, fixed reduction order, and
// reliable updates at multiples of poll_iters of its own iterations), so a
// request gives the same result alone and in the mix.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <tuple>
#include <vector>

#include "asq_batch.h"
#include "asq_internal.h"

namespace asq {
namespace {

using clk = std::chrono::steady_clock;

struct Run;

struct Request {
  uint64_t id = 0;
  int gauge_id = 0;
  int nrhs = 0;
  std::vector<double> masses;
  const double* b = nullptr;
  double* x = nullptr;
  asq_cg_params params{};
  hipEvent_t ready_ev = nullptr;  // recorded on the submitter's stream: b is ready after it
  clk::time_point t_submit, t_done;
  int state = 0;  // 0 queued, 1 running, 2 finishing (copy-out in flight), 3 done
  int rc = ASQ_OK;
  int cols_left = 0;
  int slot0 = -1;
  Run* run = nullptr;
  hipEvent_t done_ev = nullptr;
  std::vector<asq_cg_stats> stats;
  std::vector<char> col_done;
  ~Request() {
    if (ready_ev) (void)hipEventDestroy(ready_ev);
  }
};

struct Run {
  const asq_gauge* g = nullptr;
  int mode = 0;
  int cap = 0;
  int poll = 8;
  bool use_graph = true;
  bool draining = false;      // takes no new columns; destroyed once idle, freeing its stream
  size_t off = 0, bytes = 0;  // arena range
  Batch B;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev = nullptr;
  bool in_flight = false;
  ColState* pinned = nullptr;   // [cap] mirror of the device states
  ColState* staging = nullptr;  // [cap] host states uploaded when columns join
  std::vector<Request*> owner;  // per column slot
  clk::time_point t_block;
};

// First-fit allocator over the arena.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(void* b, size_t n) {
    base = (char*)b;
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = align_up(n, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n, 256);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace
}  // namespace asq

using namespace asq;

struct asq_server {
  Arena arena;
  int max_streams = 1;
  int max_cols = 1;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::vector<const asq_gauge*> gauges;
  std::list<std::unique_ptr<Run>> runs;
  uint64_t next_id = 1;
  size_t max_queue = 1 << 16;  // queued requests before serve_submit answers ASQ_EAGAIN
  bool stop = false;
  int error = ASQ_OK;
  std::thread worker;
};

namespace asq {
namespace {

// Teardown: errors are ignored, each handle is released whatever happened to
// the stream.
void destroy_run(asq_server* S, Run* r) {
  if (r->stream) (void)hipStreamSynchronize(r->stream);
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  if (r->ev) (void)hipEventDestroy(r->ev);
  if (r->stream) (void)hipStreamDestroy(r->stream);
  if (r->pinned) (void)hipHostFree(r->pinned);
  if (r->staging) (void)hipHostFree(r->staging);
  S->arena.release(r->off, r->bytes);
}

// Column slots of a run: max_cols for the largest registered field and up to
// eight times as many for smaller ones, so that runs carry similar work per
// iteration (a small field's requests would otherwise queue behind a few slots
// while its kernels wait for the GPU beside the large fields' kernels).
int run_capacity(const asq_server* S, const asq_gauge* g) {
  long hmax = 1;
  for (const asq_gauge* o : S->gauges) hmax = std::max(hmax, (long)o->geom.half);
  const long ratio = std::max(1L, std::min(8L, hmax / std::max(1L, (long)g->geom.half)));
  return (int)std::min(4096L, (long)S->max_cols * ratio);
}

int norm_poll(const asq_cg_params& p) { return p.poll_iters > 0 ? p.poll_iters : 8; }

// Whether a request may join a run: same field, precision mode and block
// shape (iterations per block and graph replay), so that its reliable updates
// fall on the iterations they would fall on in a solve of its own.
bool run_matches(const Run* r, const asq_gauge* g, const asq_cg_params& p) {
  return r->g == g && r->mode == p.mode && r->poll == norm_poll(p) && r->use_graph == (p.use_graph != 0);
}

// The key runs are grouped by: field, mode, iterations per block, graph replay.
using RunKey = std::tuple<const asq_gauge*, int, int, int>;
RunKey key_of(const Run* r) { return RunKey(r->g, r->mode, r->poll, r->use_graph ? 1 : 0); }
RunKey key_of(const asq_gauge* g, const asq_cg_params& p) {
  return RunKey(g, p.mode, norm_poll(p), p.use_graph != 0 ? 1 : 0);
}

// Create a run for (gauge, mode, block shape) if the arena and the stream
// budget allow it.  Its launch variants come from the tuner's cache (filled
// when the field was registered); nothing is timed here.
Run* make_run(asq_server* S, const asq_gauge* g, const asq_cg_params& p) {
  if ((int)S->runs.size() >= S->max_streams) return nullptr;
  int cap = run_capacity(S, g);
  size_t need = batch_bytes(g, cap, p.mode, true);
  size_t off = 0;
  if (!S->arena.alloc(need, &off)) {
    cap = S->max_cols;  // the arena decides: fall back to the base width
    need = batch_bytes(g, cap, p.mode, true);
    if (!S->arena.alloc(need, &off)) return nullptr;
  }
  std::unique_ptr<Run> r(new Run());
  r->g = g;
  r->mode = p.mode;
  r->cap = cap;
  r->poll = norm_poll(p);
  r->use_graph = p.use_graph != 0;
  r->off = off;
  r->bytes = need;
  r->owner.assign(r->cap, nullptr);
  bool ok = batch_carve(r->B, g, r->cap, p.mode, S->arena.base + off, need, nullptr, nullptr) == ASQ_OK;
  ok = ok && hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&r->pinned, r->cap * sizeof(ColState), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&r->staging, r->cap * sizeof(ColState), hipHostMallocDefault) == hipSuccess;
  if (ok) {
    // every slot starts inactive
    memset(r->staging, 0, r->cap * sizeof(ColState));
    ok = hipMemcpyAsync(r->B.st, r->staging, r->cap * sizeof(ColState), hipMemcpyHostToDevice, r->stream) ==
         hipSuccess;
  }
  if (ok && r->use_graph) ok = capture_block(r->B, r->poll, r->stream, &r->exec) == ASQ_OK;
  ok = ok && hipStreamSynchronize(r->stream) == hipSuccess;
  if (!ok) {
    destroy_run(S, r.get());
    return nullptr;
  }
  S->runs.push_back(std::move(r));
  return S->runs.back().get();
}

int free_slots(const Run* r, int n) {
  if (r->draining) return -1;
  int runlen = 0;
  for (int c = 0; c < r->cap; ++c) {
    runlen = r->owner[c] ? 0 : runlen + 1;
    if (runlen == n) return c - n + 1;
  }
  return -1;
}

// Place a queued request into a run (new columns start at this block boundary).
bool admit(asq_server* S, Request* q) {
  const asq_gauge* g = S->gauges[q->gauge_id];
  Run* run = nullptr;
  int c0 = -1;
  for (auto& r : S->runs)
    if (run_matches(r.get(), g, q->params) && (c0 = free_slots(r.get(), q->nrhs)) >= 0) {
      run = r.get();
      break;
    }
  if (!run) {
    run = make_run(S, g, q->params);
    if (!run) return false;
    c0 = free_slots(run, q->nrhs);
    if (c0 < 0) return false;
  }
  const size_t half = (size_t)g->geom.half;
  hipStream_t s = run->stream;
  Batch& B = run->B;
  asq_cg_params p = q->params;
  p.mode = run->mode;
  // per-column constants, then b into the slots, then the init kernels
  Batch tmp = B;
  tmp.ncol = q->nrhs;
  init_states(tmp, q->masses.data(), &p, run->staging + c0, nullptr);
  bool ok = hipMemcpyAsync(B.st + c0, run->staging + c0, q->nrhs * sizeof(ColState), hipMemcpyHostToDevice, s) ==
            hipSuccess;
  // b as the submitter's stream left it, relayout into the slots' native layout
  ok = ok && hipStreamWaitEvent(s, q->ready_ev, 0) == hipSuccess;
  ok = ok && relayout(VEC_F64, true, q->nrhs, (int)half, q->b, B.b + (size_t)c0 * half * 6, s) == ASQ_OK;
  ok = ok && enqueue_init(B, c0, q->nrhs, s) == ASQ_OK;
  if (!ok) {
    q->rc = ASQ_EHIP;
    q->state = 3;
    q->t_done = clk::now();
    return true;
  }
  for (int c = 0; c < q->nrhs; ++c) run->owner[c0 + c] = q;
  q->run = run;
  q->slot0 = c0;
  q->cols_left = q->nrhs;
  q->stats.assign(q->nrhs, asq_cg_stats{});
  q->col_done.assign(q->nrhs, 0);
  q->state = 1;
  return true;
}

// A HIP call on a run's stream failed: every request running in it ends with
// ASQ_EHIP, and the run takes no new columns and is destroyed once idle.
void fail_run(Run* r) {
  for (int c = 0; c < r->cap; ++c) {
    Request* q = r->owner[c];
    if (!q) continue;
    if (q->state == 1) {
      q->rc = ASQ_EHIP;
      q->state = 3;
      q->t_done = clk::now();
    }
    r->owner[c] = nullptr;
  }
  r->in_flight = false;
  r->draining = true;
}

void launch_block(Run* r) {
  bool ok = r->exec ? hipGraphLaunch(r->exec, r->stream) == hipSuccess
                    : enqueue_block(r->B, r->poll, r->stream) == ASQ_OK;
  ok = ok && hipMemcpyAsync(r->pinned, r->B.st, r->cap * sizeof(ColState), hipMemcpyDeviceToHost, r->stream) ==
                 hipSuccess;
  ok = ok && hipEventRecord(r->ev, r->stream) == hipSuccess;
  if (!ok) {
    fail_run(r);
    return;
  }
  r->in_flight = true;
  r->t_block = clk::now();
}

// Retire finished columns of a run whose block has completed.  A finished
// column keeps its slot (its x is still in the batch) until every column of
// its request is done; then x is copied out and all the request's slots are
// released together (later work on this stream is ordered after the copy).
void harvest(asq_server* S, Run* r) {
  const size_t half = (size_t)r->g->geom.half;
  for (int c = 0; c < r->cap; ++c) {
    Request* q = r->owner[c];
    if (!q || q->state != 1) continue;
    const int k = c - q->slot0;
    if (q->col_done[k]) continue;
    const ColState& st = r->pinned[c];
    if (st.active) continue;
    int worst = ASQ_OK;
    Batch one = r->B;
    one.ncol = 1;
    fill_stats(one, &st, 0.0, &q->stats[k], &worst);
    if (worst != ASQ_OK && (q->rc == ASQ_OK || worst == ASQ_ENAN)) q->rc = worst;
    q->col_done[k] = 1;
    if (--q->cols_left == 0) {
      bool ok = relayout(VEC_F64, false, q->nrhs, (int)half, r->B.x + (size_t)q->slot0 * half * 6, q->x,
                         r->stream) == ASQ_OK;
      ok = ok && hipEventCreateWithFlags(&q->done_ev, hipEventDisableTiming) == hipSuccess;
      ok = ok && hipEventRecord(q->done_ev, r->stream) == hipSuccess;
      for (int j = 0; j < q->nrhs; ++j) r->owner[q->slot0 + j] = nullptr;
      if (ok) {
        q->state = 2;
      } else {
        // without a recorded event the copy cannot be waited for: end the request here
        if (q->done_ev) (void)hipEventDestroy(q->done_ev);
        q->done_ev = nullptr;
        q->rc = ASQ_EHIP;
        q->state = 3;
        q->t_done = clk::now();
      }
    }
  }
  (void)S;
}

void finish_copies(asq_server* S) {
  for (auto& kv : S->reqs) {
    Request* q = kv.second.get();
    if (q->state != 2) continue;
    const hipError_t e = hipEventQuery(q->done_ev);
    if (e != hipErrorNotReady) {
      if (e != hipSuccess) q->rc = ASQ_EHIP;
      (void)hipEventDestroy(q->done_ev);
      q->done_ev = nullptr;
      q->t_done = clk::now();
      const double secs = std::chrono::duration<double>(q->t_done - q->t_submit).count();
      for (auto& st : q->stats) st.seconds = secs;
      q->state = 3;
    }
  }
}

bool run_idle(const Run* r) {
  for (auto* o : r->owner)
    if (o) return false;
  return true;
}

int used_slots(const Run* r) {
  int n = 0;
  for (auto* o : r->owner) n += o != nullptr;
  return n;
}

// Every stream is taken and a queued request's field has no run at all: let a
// field that holds two or more runs give one up (the least occupied stops
// taking columns and is destroyed once its columns are done), so that one busy
// field cannot starve the others.  At most one run drains at a time.
void make_room(asq_server* S, const RunKey& k) {
  if ((int)S->runs.size() < S->max_streams) return;
  std::map<RunKey, int> per_field;
  for (auto& r : S->runs) {
    if (r->draining) return;
    per_field[key_of(r.get())] += 1;
  }
  if (per_field.count(k)) return;
  Run* victim = nullptr;
  for (auto& r : S->runs)
    if (per_field[key_of(r.get())] >= 2 && (!victim || used_slots(r.get()) < used_slots(victim))) victim = r.get();
  if (victim) victim->draining = true;
}

void worker_main(asq_server* S) {
  // the device was current in serve_create, so this cannot fail on it
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    // admission at block boundaries: only runs that are not in flight take new columns
    for (auto it = S->queue.begin(); it != S->queue.end();) {
      Request* q = *it;
      bool placed = false;
      bool blocked_by_flight = false;
      const asq_gauge* g = S->gauges[q->gauge_id];
      for (auto& r : S->runs)
        if (run_matches(r.get(), g, q->params) && r->in_flight && free_slots(r.get(), q->nrhs) >= 0)
          blocked_by_flight = true;
      if (!blocked_by_flight) placed = admit(S, q);
      if (!placed && !blocked_by_flight) make_room(S, key_of(g, q->params));
      if (placed) it = S->queue.erase(it);
      else ++it;
    }
    bool any_flight = false;
    for (auto& r : S->runs) {
      if (!r->in_flight && !run_idle(r.get())) launch_block(r.get());
      any_flight |= r->in_flight;
    }
    finish_copies(S);
    // An idle run gives up its stream and arena range only to a queued request
    // whose field has no run to join; otherwise it stays for its own field.
    bool need_run = false;
    for (Request* q : S->queue) {
      bool has = false;
      for (auto& r : S->runs) has |= !r->draining && run_matches(r.get(), S->gauges[q->gauge_id], q->params);
      need_run |= !has;
    }
    if (need_run) {
      // While the streams cover every field in use (gauge and mode, running or
      // queued), a field's only run is kept even when idle (small fields would
      // otherwise lose their stream between requests); streams for a new field
      // come from drained extra runs.
      std::set<RunKey> fields;
      for (auto& r : S->runs) fields.insert(key_of(r.get()));
      for (Request* q : S->queue) fields.insert(key_of(S->gauges[q->gauge_id], q->params));
      const bool keep_last = (int)fields.size() <= S->max_streams;
      for (auto it = S->runs.begin(); it != S->runs.end();) {
        Run* r = it->get();
        int same = 0;
        for (auto& o : S->runs) same += !o->draining && key_of(o.get()) == key_of(r);
        const bool last_of_field = !r->draining && same == 1;
        if (!r->in_flight && run_idle(r) && !(keep_last && last_of_field)) {
          bool copies_pending = false;
          for (auto& kv : S->reqs)
            if (kv.second->state == 2 && kv.second->run == r) copies_pending = true;
          if (!copies_pending) {
            destroy_run(S, r);
            it = S->runs.erase(it);
            continue;
          }
        }
        ++it;
      }
    }
    bool copies = false;
    for (auto& kv : S->reqs) copies |= kv.second->state == 2;
    if (S->stop && S->queue.empty() && !any_flight && !copies) break;
    if (!any_flight && S->queue.empty() && !copies) {
      S->cv.wait(lk);
      continue;
    }
    // poll the in-flight blocks without holding the lock
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
    for (auto& r : S->runs) {
      if (!r->in_flight) continue;
      const hipError_t e = hipEventQuery(r->ev);
      if (e == hipSuccess) {
        r->in_flight = false;
        harvest(S, r.get());
      } else if (e != hipErrorNotReady) {
        fail_run(r.get());
      }
    }
  }
  for (auto& r : S->runs) destroy_run(S, r.get());
  S->runs.clear();
}

}  // namespace
}  // namespace asq

extern "C" int serve_create(void* arena_dev, size_t arena_bytes, int max_streams, int max_cols, asq_server** out) {
  if (!out || !arena_dev || arena_bytes == 0 || max_streams < 1 || max_streams > 64 || max_cols < 1 ||
      max_cols > 4096 || ((uintptr_t)arena_dev & 255)) {
    set_last_error("serve_create: invalid arguments (arena 256-byte aligned, 1 <= max_streams <= 64)");
    return ASQ_EINVAL;
  }
  int device = 0;
  ASQ_HIP_TRY(hipGetDevice(&device));
  asq_server* S = new asq_server();
  S->arena.init(arena_dev, arena_bytes);
  S->max_streams = max_streams;
  S->max_cols = max_cols;
  S->device = device;
  // ASQ_SERVE_MAX_QUEUE=<n>: a shorter queue (tests force ASQ_EAGAIN with it)
  if (const char* e = getenv("ASQ_SERVE_MAX_QUEUE")) {
    const long n = atol(e);
    if (n > 0) S->max_queue = (size_t)n;
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return ASQ_OK;
}

namespace asq {
namespace {

// Tune the Dslash launches of every run shape the registered fields can get
// (each precision mode a field keeps links for, at its run width and at the
// fallback width), on scratch taken from the arena, while no run exists, so
// the timings see an idle device.  Runs later take the tuned variants from the
// tuner's cache without timing anything.  Called with S->mu held.
void tune_fields(asq_server* S) {
  if (!S->runs.empty()) {
    if (log_enabled()) fprintf(stderr, "[asq] serve: runs exist, launch variants not tuned\n");
    return;
  }
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  for (const asq_gauge* g : S->gauges)
    for (int mode = ASQ_MODE_F64; mode <= ASQ_MODE_MIXED16; ++mode) {
      asq_cg_params p{};
      p.mode = mode;
      p.tol = 1;
      p.maxiter = 1;
      if (check_params(g, &p)) continue;  // the field keeps no links for this mode
      for (int w : {run_capacity(S, g), S->max_cols}) {
        const size_t need = batch_bytes(g, w, mode, true);
        size_t off = 0;
        if (!S->arena.alloc(need, &off)) continue;
        Batch B;
        if (batch_carve(B, g, w, mode, S->arena.base + off, need, nullptr, nullptr) == ASQ_OK)
          (void)batch_tune(B, st, true);
        (void)hipStreamSynchronize(st);
        S->arena.release(off, need);
      }
    }
  (void)hipStreamDestroy(st);
}

}  // namespace
}  // namespace asq

extern "C" int serve_register_gauge(asq_server* S, const asq_gauge* g, int* gauge_id) {
  if (!S || !g || !gauge_id) return ASQ_EINVAL;
  if (!g->links[LINK_F64_R18]) {
    set_last_error("serve_register_gauge: the gauge field must keep FP64 links");
    return ASQ_EINVAL;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->gauges.push_back(g);
  *gauge_id = (int)S->gauges.size() - 1;
  tune_fields(S);
  return ASQ_OK;
}

extern "C" int serve_submit(asq_server* S, int gauge_id, int nrhs, const double* masses, const double* b_dev,
                            double* x_dev, const asq_cg_params* params, uint64_t* ticket, void* hip_stream) {
  if (!S || !masses || !b_dev || !x_dev || !params || !ticket || nrhs <= 0) return ASQ_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  if (gauge_id < 0 || gauge_id >= (int)S->gauges.size()) return ASQ_EINVAL;
  const asq_gauge* g = S->gauges[gauge_id];
  if (check_params(g, params)) {
    set_last_error("serve_submit: invalid parameters");
    return ASQ_EINVAL;
  }
  for (int c = 0; c < nrhs; ++c)
    if (!(masses[c] > 0) || !isfinite(masses[c])) return ASQ_EINVAL;
  if (((uintptr_t)b_dev & 15) || ((uintptr_t)x_dev & 15)) return ASQ_EINVAL;
  const size_t vbytes = (size_t)nrhs * g->geom.half * 48;
  if (ranges_overlap(b_dev, vbytes, x_dev, vbytes)) return ASQ_EINVAL;
  if (nrhs > S->max_cols || batch_bytes(g, S->max_cols, params->mode, true) > S->arena.size) {
    set_last_error("serve_submit: request can never fit (nrhs > max_cols or a batch exceeds the arena)");
    return ASQ_ENOMEM;
  }
  if (S->queue.size() >= S->max_queue) {
    set_last_error("serve_submit: queue full");
    return ASQ_EAGAIN;
  }
  std::unique_ptr<Request> q(new Request());
  // the server reads b after the work enqueued so far on the submitter's stream
  if (hipEventCreateWithFlags(&q->ready_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(q->ready_ev, (hipStream_t)hip_stream) != hipSuccess) {
    set_last_error("serve_submit: could not record an event on the stream");
    return ASQ_EHIP;
  }
  q->id = S->next_id++;
  q->gauge_id = gauge_id;
  q->nrhs = nrhs;
  q->masses.assign(masses, masses + nrhs);
  q->b = b_dev;
  q->x = x_dev;
  q->params = *params;
  q->t_submit = clk::now();
  *ticket = q->id;
  S->queue.push_back(q.get());
  S->reqs[q->id] = std::move(q);
  S->cv.notify_one();
  return ASQ_OK;
}

extern "C" int serve_poll(asq_server* S, uint64_t ticket, asq_cg_stats* per_rhs, double* latency_s) {
  if (!S) return ASQ_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return ASQ_EINVAL;
  Request* q = it->second.get();
  if (q->state != 3) return ASQ_PENDING;
  if (per_rhs)
    for (int c = 0; c < q->nrhs; ++c) per_rhs[c] = q->stats[c];
  if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_submit).count();
  const int rc = q->rc;
  S->reqs.erase(it);
  return rc;
}

extern "C" int serve_destroy(asq_server* S) {
  if (!S) return ASQ_EINVAL;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_one();
  }
  S->worker.join();
  delete S;
  return ASQ_OK;
}
