// Serving runtime: admission of independent sketch / RSVD / Nystrom jobs against a
// device arena (the HBM budget), a plan cache inside that arena, and an
// event-driven executor: every admitted job is a coroutine on one of a few
// HIP streams, resumed by the thread that calls the server whenever the event
// it waits on has completed (continuous batching without worker threads).
// The host-only test executor runs jobs as sleeps on worker threads instead.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <optional>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/bsrht_serve.h"
#include "common.h"
#include "task.h"

namespace bsrht {
namespace {

constexpr size_t kAlign = 256;
constexpr int kBackfillWindow = 8;       // younger jobs considered past the oldest
constexpr double kMaxBypassSeconds = 0.1;  // after this, nothing passes the oldest
constexpr int kMaxWorkers = 64;
constexpr size_t kStagingHalf = 64 * 1024;  // pinned bytes per direction per stream slot
constexpr double kPollSleep = 20e-6;        // seconds between executor passes while waiting
constexpr int kBatchJobs = BSRHT_BATCH_MAX;    // small sketch jobs fused into one launch
constexpr int64_t kBatchJobBytes = 64 << 20;   // A of at most this many bytes is "small"

size_t round_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over byte offsets [0, size) with coalescing.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        bytes += prev->second;
        free_.erase(prev);
      }
    }
    next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      free_.erase(next);
    }
    free_[off] = bytes;
  }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used_ = 0;
};

using PlanKey = std::tuple<int64_t, int64_t, int64_t, uint64_t, int, int>;

struct PlanEntry {
  enum State { PENDING, READY, FAILED };
  PlanKey key;
  bsrht_plan_t plan = nullptr;
  size_t off = 0, bytes = 0;
  int refs = 0;
  State state = PENDING;
  int status = BSRHT_OK;
  uint64_t last_use = 0;
};

struct Job {
  bsrht_job_t j;
  size_t ws_off = 0, ws_bytes = 0;
  bool has_ws = false;
  PlanEntry *pe = nullptr;
  double t_submit = 0.0, t_start = 0.0;
  int64_t held = 0;
};

// Plan-shaped descriptor without tables: enough for the workspace queries.
bsrht_plan_s shape_of(const bsrht_job_t &j) {
  bsrht_plan_s s{};
  s.n = j.n;
  s.p = j.p;
  s.l = j.l;
  s.r = j.n / j.p;
  int lg = 0;
  while ((int64_t(1) << lg) < s.r) ++lg;
  s.log2r = lg;
  s.rp = int64_t(1) << lg;
  s.seed = j.seed;
  s.sampling = j.sampling;
  s.precision = j.precision;
  s.d_words = (j.p * s.rp + 31) / 32;
  s.dt_words = (j.l + 31) / 32;
  return s;
}

size_t workspace_of(const bsrht_job_t &j) {
  bsrht_plan_s s = shape_of(j);
  if (j.kind == BSRHT_JOB_SKETCH) return bsrht_apply_workspace(&s, j.m);
  if (j.kind == BSRHT_JOB_NYSTROM) return nystrom_workspace(&s, j.k);
  return rsvd_workspace(&s, j.m, j.k);
}

bool valid_job(const bsrht_job_t &j, bool fake) {
  if (j.kind != BSRHT_JOB_SKETCH && j.kind != BSRHT_JOB_RSVD && j.kind != BSRHT_JOB_NYSTROM)
    return false;
  if (j.kind == BSRHT_JOB_NYSTROM && j.m != j.n) return false;
  if (j.m < 1 || j.m > INT32_MAX || bsrht_plan_bytes(j.n, j.p, j.l) == 0) return false;
  if (j.sampling != BSRHT_WITH_REPLACEMENT && j.sampling != BSRHT_WITHOUT_REPLACEMENT)
    return false;
  if (j.sampling == BSRHT_WITHOUT_REPLACEMENT && j.l > shape_of(j).rp) return false;
  if (j.precision != BSRHT_FP32 && j.precision != BSRHT_SPLIT_BF16) return false;
  if (j.lda < j.m) return false;
  if (j.kind == BSRHT_JOB_SKETCH && j.ldy < j.m) return false;
  if (j.kind != BSRHT_JOB_SKETCH && j.k < 1) return false;
  if (fake) return true;
  if (!j.A) return false;
  if (j.kind == BSRHT_JOB_SKETCH) return j.Y != nullptr;
  if (j.kind == BSRHT_JOB_NYSTROM) return j.U && j.S && j.info;
  return j.U && j.S && j.V && j.info;
}

// A job whose sketch may run fused with other small ones in one batched,
// graph-replayed launch (bsrht_apply_batch): FP32, blocks of >= 64 rows, A
// of at most kBatchJobBytes.
bool batchable(const bsrht_job_t &j) {
  const int64_t r = j.n / j.p;
  return j.kind == BSRHT_JOB_SKETCH && j.precision == BSRHT_FP32 && r >= 64 &&
         (r & (r - 1)) == 0 && j.n * j.m * 4 <= kBatchJobBytes;
}

// The work of one job on its slot's stream, ending when the stream has
// finished it.
Task sketch_job(DevCtx &ctx, bsrht_plan_t plan, const bsrht_job_t j, void *ws, size_t ws_bytes) {
  const int st = bsrht_apply(plan, j.A, j.m, j.lda, j.Y, j.ldy, ws, ws_bytes, ctx.s);
  if (st != BSRHT_OK) co_return st;
  co_return co_await drained(ctx);
}

// Several small sketch jobs as one batched launch on the slot's stream.
Task batch_job(DevCtx &ctx, std::vector<bsrht_apply_item_t> items, void *table,
               size_t table_bytes) {
  const int st =
      bsrht_apply_batch(items.data(), (int)items.size(), table, table_bytes, ctx.s);
  if (st != BSRHT_OK) co_return st;
  co_return co_await drained(ctx);
}

Task rsvd_job(DevCtx &ctx, bsrht_plan_t plan, const bsrht_job_t j, void *ws, size_t ws_bytes) {
  const int st = co_await rsvd_task(ctx, plan, j.A, j.m, j.lda, j.k, j.U, j.S, j.V, j.info, ws,
                                    ws_bytes);
  if (st != BSRHT_OK) co_return st;
  co_return co_await drained(ctx);
}

Task nystrom_job(DevCtx &ctx, bsrht_plan_t plan, const bsrht_job_t j, void *ws,
                 size_t ws_bytes) {
  const int st = co_await nystrom_task(ctx, plan, j.A, j.lda, j.k, j.U, j.S, j.info, ws,
                                       ws_bytes, false);
  if (st != BSRHT_OK) co_return st;
  co_return co_await drained(ctx);
}

struct Slot {
  DevCtx ctx;
  Job *job = nullptr;
  std::vector<Job *> batch;  // the jobs of a batched launch (job == nullptr then)
  size_t table_off = 0;      // the slot's batch descriptor table in the arena
  bool has_table = false;
  std::optional<Task> task;
  bool busy() const { return job != nullptr || !batch.empty(); }
};

}  // namespace
}  // namespace bsrht

using namespace bsrht;

struct bsrht_server_s {
  bool fake = false;
  bool batching = true;  // small sketch jobs may run as batched launches
  double sec_per_gb = 0.0;
  char *base = nullptr;
  size_t arena_bytes = 0;
  int device = 0;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;  // host-only executor
  Arena arena;
  std::deque<Job *> queue;  // submitted, not admitted (arrival order)
  std::deque<Job *> ready;  // admitted, not yet taken by a worker
  int running = 0;
  bool stop = false;
  std::deque<bsrht_job_result_t> results;
  std::map<PlanKey, PlanEntry *> plans;
  uint64_t tick = 0;
  bsrht_server_stats_t st{};
  int nworkers = 0;                 // concurrent jobs: worker threads or stream slots
  std::vector<std::thread> threads;  // host-only executor
  std::vector<Slot> slots;           // GPU executor

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Frees the least recently used plan that no admitted job holds.
  bool evict_one() {
    PlanEntry *victim = nullptr;
    for (auto &kv : plans) {
      PlanEntry *pe = kv.second;
      if (pe->refs == 0 && (pe->state == PlanEntry::READY || pe->state == PlanEntry::FAILED) &&
          (!victim || pe->last_use < victim->last_use))
        victim = pe;
    }
    if (!victim) return false;
    drop_plan(victim);
    ++st.plan_evictions;
    return true;
  }

  void drop_plan(PlanEntry *pe) {
    if (pe->plan) bsrht_plan_destroy(pe->plan);
    arena.release(pe->off, pe->bytes);
    plans.erase(pe->key);
    delete pe;
  }

  // Reserves the job's workspace and, on a cache miss, its plan's tables.
  bool reserve(Job *jb) {
    const bsrht_job_t &j = jb->j;
    const PlanKey key{j.n, j.p, j.l, j.seed, j.sampling, j.precision};
    auto it = plans.find(key);
    PlanEntry *pe = it == plans.end() ? nullptr : it->second;
    const size_t ws = workspace_of(j);
    const size_t tb = pe ? 0 : bsrht_plan_bytes(j.n, j.p, j.l);
    for (;;) {
      size_t ws_off = 0, tb_off = 0;
      bool ok = true;
      if (ws && !arena.alloc(ws, &ws_off)) ok = false;
      if (ok && tb && !arena.alloc(tb, &tb_off)) {
        if (ws) arena.release(ws_off, ws);
        ok = false;
      }
      if (ok) {
        if (!pe) {
          pe = new PlanEntry;
          pe->key = key;
          pe->off = tb_off;
          pe->bytes = tb;
          plans[key] = pe;
          ++st.plan_misses;
        } else {
          ++st.plan_hits;
        }
        ++pe->refs;
        pe->last_use = ++tick;
        jb->pe = pe;
        jb->ws_off = ws_off;
        jb->ws_bytes = ws;
        jb->has_ws = ws != 0;
        jb->held = (int64_t)(round_up(ws) + round_up(tb));
        return true;
      }
      if (!evict_one()) return false;
      // the evicted plan may have been this job's: look it up again
      it = plans.find(key);
      pe = it == plans.end() ? nullptr : it->second;
      if (!pe && tb == 0) return reserve(jb);
    }
  }

  // Admits waiting jobs while a worker is free (called with mu held).  The
  // GPU executor also admits up to kBatchJobs small sketch jobs beyond that,
  // which a free slot then runs as one batched launch.
  void admit() {
    while (!queue.empty()) {
      const int busy = (int)ready.size() + running;
      const bool room = busy < nworkers;
      if (!room && (fake || !batching || busy >= nworkers + kBatchJobs)) break;
      const bool overdue = now() - queue.front()->t_submit > kMaxBypassSeconds;
      const int window = overdue ? 1 : std::min<int>((int)queue.size(), kBackfillWindow);
      bool admitted = false;
      for (int i = 0; i < window; ++i) {
        Job *jb = queue[(size_t)i];
        if (!room && !batchable(jb->j)) continue;
        if (!reserve(jb)) continue;
        if (i > 0) ++st.backfilled;
        queue.erase(queue.begin() + i);
        ready.push_back(jb);
        st.peak_arena_bytes = std::max<int64_t>(st.peak_arena_bytes, (int64_t)arena.used());
        admitted = true;
        break;
      }
      if (!admitted) break;
    }
    cv_work.notify_all();
  }

  // Releases a finished job's arena bytes and plan reference and records its
  // result (mu held).
  void retire(Job *jb, int rc, double t_done) {
    PlanEntry *pe = jb->pe;
    if (jb->has_ws) arena.release(jb->ws_off, jb->ws_bytes);
    --pe->refs;
    pe->last_use = ++tick;
    if (pe->state == PlanEntry::FAILED && pe->refs == 0) drop_plan(pe);
    bsrht_job_result_t r;
    r.id = jb->j.id;
    r.status = rc;
    r.arena_bytes = jb->held;
    r.t_submit = jb->t_submit;
    r.t_start = jb->t_start;
    r.t_done = t_done;
    results.push_back(r);
    delete jb;
    --running;
    ++st.completed;
  }

  // ---- host-only executor: worker threads that sleep in place of work ----
  void worker() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || !ready.empty(); });
      if (ready.empty()) return;  // stop requested and nothing left
      Job *jb = ready.front();
      ready.pop_front();
      ++running;
      st.peak_running = std::max(st.peak_running, running);
      jb->t_start = now();
      if (jb->pe->state == PlanEntry::PENDING) jb->pe->state = PlanEntry::READY;
      lk.unlock();
      const double secs = sec_per_gb * 4.0 * (double)jb->j.n * (double)jb->j.m / 1e9;
      std::this_thread::sleep_for(std::chrono::duration<double>(secs));
      lk.lock();
      retire(jb, BSRHT_OK, now());
      admit();
      cv_done.notify_all();
    }
  }

  // ---- GPU executor ----
  // Marks the job running and builds its plan on the slot's stream when it is
  // not cached yet; false (job retired) when the plan cannot be built.
  bool begin_job(Slot &sl, Job *jb) {
    ++running;
    st.peak_running = std::max(st.peak_running, running);
    jb->t_start = now();
    PlanEntry *pe = jb->pe;
    if (pe->state == PlanEntry::PENDING) {
      const auto &[n, p, l, seed, sampling, precision] = pe->key;
      int rc = bsrht_plan(n, p, l, seed, sampling, precision, base + pe->off, pe->bytes,
                          sl.ctx.s, &pe->plan);
      if (rc == BSRHT_OK && hipStreamSynchronize(sl.ctx.s) != hipSuccess) rc = BSRHT_EDEVICE;
      pe->state = rc == BSRHT_OK ? PlanEntry::READY : PlanEntry::FAILED;
      pe->status = rc;
    }
    if (pe->state == PlanEntry::FAILED) {
      retire(jb, pe->status, now());
      return false;
    }
    return true;
  }

  void start_batch(Slot &sl, std::vector<Job *> &jobs) {
    std::vector<bsrht_apply_item_t> items;
    for (Job *jb : jobs) {
      if (!begin_job(sl, jb)) continue;
      sl.batch.push_back(jb);
      const bsrht_job_t &j = jb->j;
      bsrht_apply_item_t it;
      it.plan = jb->pe->plan;
      it.A = j.A;
      it.m = j.m;
      it.lda = j.lda;
      it.Y = j.Y;
      it.ldy = j.ldy;
      it.ws = jb->has_ws ? base + jb->ws_off : nullptr;
      it.ws_bytes = jb->ws_bytes;
      items.push_back(it);
    }
    if (items.empty()) return;
    ++st.batches;
    st.batched_jobs += (int64_t)items.size();
    sl.task.emplace(batch_job(sl.ctx, std::move(items), base + sl.table_off,
                              bsrht_batch_table_bytes()));
    sl.task->start();
  }

  void start_job(Slot &sl, Job *jb) {
    if (!begin_job(sl, jb)) return;
    sl.job = jb;
    PlanEntry *pe = jb->pe;
    void *ws = jb->has_ws ? base + jb->ws_off : nullptr;
    if (jb->j.kind == BSRHT_JOB_SKETCH)
      sl.task.emplace(sketch_job(sl.ctx, pe->plan, jb->j, ws, jb->ws_bytes));
    else if (jb->j.kind == BSRHT_JOB_NYSTROM)
      sl.task.emplace(nystrom_job(sl.ctx, pe->plan, jb->j, ws, jb->ws_bytes));
    else
      sl.task.emplace(rsvd_job(sl.ctx, pe->plan, jb->j, ws, jb->ws_bytes));
    sl.task->start();  // runs until its first wait on the device
  }

  void finish_slot(Slot &sl, int rc) {
    Job *jb = sl.job;
    sl.job = nullptr;
    sl.task.reset();
    const double t = now();
    if (jb) retire(jb, rc, t);
    for (Job *b : sl.batch) retire(b, rc, t);
    sl.batch.clear();
  }

  // One executor pass: resume jobs whose awaited event has completed, retire
  // finished jobs, admit and start waiting ones (mu held).  Repeats while it
  // makes progress.
  void pump() {
    for (bool moved = true; moved;) {
      moved = false;
      for (Slot &sl : slots) {
        if (!sl.busy()) continue;
        if (!sl.task->done()) {
          const hipError_t q = hipEventQuery(sl.ctx.ev);
          if (q == hipErrorNotReady) continue;
          if (q != hipSuccess) {
            finish_slot(sl, BSRHT_EDEVICE);
            moved = true;
            continue;
          }
          sl.ctx.resume_point.resume();
          moved = true;
        }
        if (sl.task->done()) {
          finish_slot(sl, sl.task->status());
          moved = true;
        }
      }
      admit();
      for (Slot &sl : slots) {
        if (sl.busy() || ready.empty()) continue;
        if (batching && sl.has_table && batchable(ready.front()->j)) {
          // the small sketch jobs among the ready ones, in order
          std::vector<Job *> b;
          for (auto it = ready.begin(); it != ready.end() && (int)b.size() < kBatchJobs;) {
            if (batchable((*it)->j)) {
              b.push_back(*it);
              it = ready.erase(it);
            } else {
              ++it;
            }
          }
          if (b.size() >= 2) {
            start_batch(sl, b);
            moved = true;
            continue;
          }
          ready.push_front(b[0]);
        }
        Job *jb = ready.front();
        ready.pop_front();
        start_job(sl, jb);
        moved = true;
      }
    }
  }

  int start(int workers) {
    nworkers = workers;
    t0 = std::chrono::steady_clock::now();
    arena.reset(arena_bytes);
    if (fake) {
      for (int w = 0; w < workers; ++w) threads.emplace_back(&bsrht_server_s::worker, this);
      return BSRHT_OK;
    }
    if (hipGetDevice(&device) != hipSuccess) return BSRHT_EDEVICE;
    slots.resize((size_t)workers);
    for (Slot &sl : slots) {
      void *pin = nullptr;
      if (hipStreamCreateWithFlags(&sl.ctx.s, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.ctx.ev, hipEventDisableTiming) != hipSuccess ||
          hipHostMalloc(&pin, 2 * kStagingHalf, hipHostMallocDefault) != hipSuccess)
        return BSRHT_EDEVICE;
      sl.ctx.blocking = false;
      sl.ctx.pinned = static_cast<char *>(pin);
      sl.ctx.half_bytes = kStagingHalf;
      // a slot without room for a descriptor table runs small jobs one by one
      sl.has_table = arena.alloc(bsrht_batch_table_bytes(), &sl.table_off);
    }
    return BSRHT_OK;
  }

  void release_device() {
    if (!slots.empty()) (void)hipSetDevice(device);
    for (Slot &sl : slots) {
      sl.task.reset();
      // the batched launches of this slot's table (graph, staging, event)
      if (sl.has_table) (void)bsrht_batch_table_release(base + sl.table_off);
      if (sl.ctx.pinned) (void)hipHostFree(sl.ctx.pinned);
      if (sl.ctx.ev) (void)hipEventDestroy(sl.ctx.ev);
      if (sl.ctx.s) (void)hipStreamDestroy(sl.ctx.s);
    }
    slots.clear();
  }
};

namespace {

int create(bool fake, void *arena, size_t arena_bytes, int workers, double sec_per_gb,
           bsrht_server_t *out) {
  if (!out) return BSRHT_EINVAL;
  *out = nullptr;
  if (workers < 1 || workers > kMaxWorkers || arena_bytes == 0) return BSRHT_EINVAL;
  if (!fake && (!arena || ((uintptr_t)arena % kAlign) != 0)) return BSRHT_EINVAL;
  bsrht_server_s *srv = new (std::nothrow) bsrht_server_s;
  if (!srv) return BSRHT_ENOMEM;
  srv->fake = fake;
  srv->sec_per_gb = sec_per_gb;
  srv->base = static_cast<char *>(arena);
  srv->arena_bytes = arena_bytes & ~(kAlign - 1);
  const int rc = srv->start(workers);
  if (rc != BSRHT_OK) {
    srv->release_device();
    delete srv;
    return rc;
  }
  *out = srv;
  return BSRHT_OK;
}

}  // namespace

extern "C" {

size_t bsrht_job_bytes(const bsrht_job_t *job) {
  if (!job || !valid_job(*job, true)) return 0;
  return round_up(workspace_of(*job)) + round_up(bsrht_plan_bytes(job->n, job->p, job->l));
}

int bsrht_server_create(void *arena, size_t arena_bytes, int streams, bsrht_server_t *out) {
  return create(false, arena, arena_bytes, streams, 0.0, out);
}

int bsrht_server_create_fake(size_t arena_bytes, int workers, double seconds_per_gb,
                             bsrht_server_t *out) {
  if (!(seconds_per_gb >= 0.0)) return BSRHT_EINVAL;
  return create(true, nullptr, arena_bytes, workers, seconds_per_gb, out);
}

int bsrht_server_submit(bsrht_server_t srv, const bsrht_job_t *job) {
  if (!srv || !job || !valid_job(*job, srv->fake)) {
    if (srv) {
      std::lock_guard<std::mutex> lk(srv->mu);
      ++srv->st.rejected;
    }
    return BSRHT_EINVAL;
  }
  if (bsrht_job_bytes(job) > srv->arena_bytes) {
    std::lock_guard<std::mutex> lk(srv->mu);
    ++srv->st.rejected;
    return BSRHT_ENOMEM;
  }
  Job *jb = new (std::nothrow) Job;
  if (!jb) return BSRHT_ENOMEM;
  jb->j = *job;
  std::lock_guard<std::mutex> lk(srv->mu);
  jb->t_submit = srv->now();
  srv->queue.push_back(jb);
  ++srv->st.submitted;
  srv->admit();
  if (!srv->fake) srv->pump();
  return BSRHT_OK;
}

int bsrht_server_submit_many(bsrht_server_t srv, const bsrht_job_t *jobs, int count,
                             int *accepted) {
  if (!srv || count < 0 || (count > 0 && !jobs) || !accepted) return BSRHT_EINVAL;
  *accepted = 0;
  std::vector<Job *> made;
  int rc = BSRHT_OK;
  for (int i = 0; i < count; ++i) {
    const bsrht_job_t &j = jobs[i];
    if (!valid_job(j, srv->fake)) {
      rc = BSRHT_EINVAL;
    } else if (bsrht_job_bytes(&j) > srv->arena_bytes) {
      rc = BSRHT_ENOMEM;
    } else {
      Job *jb = new (std::nothrow) Job;
      if (!jb) {
        rc = BSRHT_ENOMEM;
      } else {
        jb->j = j;
        made.push_back(jb);
        continue;
      }
    }
    break;  // the first rejected job stops the call
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (rc != BSRHT_OK) ++srv->st.rejected;
  const double t = srv->now();
  for (Job *jb : made) {
    jb->t_submit = t;
    srv->queue.push_back(jb);
    ++srv->st.submitted;
  }
  *accepted = (int)made.size();
  srv->admit();
  if (!srv->fake) srv->pump();
  return rc;
}

int bsrht_server_poll(bsrht_server_t srv, bsrht_job_result_t *out, int max, double timeout_s,
                      int *count) {
  if (!srv || !count || max < 0 || (max > 0 && !out)) return BSRHT_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->fake) {
    if (srv->results.empty() && timeout_s > 0.0)
      srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                            [&] { return !srv->results.empty(); });
  } else {
    const double until = srv->now() + std::max(timeout_s, 0.0);
    for (;;) {
      srv->pump();
      if (!srv->results.empty() || srv->now() >= until) break;
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::duration<double>(kPollSleep));
      lk.lock();
    }
  }
  int c = 0;
  while (c < max && !srv->results.empty()) {
    out[c++] = srv->results.front();
    srv->results.pop_front();
  }
  *count = c;
  return BSRHT_OK;
}

int bsrht_server_drain(bsrht_server_t srv) {
  if (!srv) return BSRHT_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->fake) {
    srv->cv_done.wait(lk, [&] { return srv->st.completed == srv->st.submitted; });
    return BSRHT_OK;
  }
  for (;;) {
    srv->pump();
    if (srv->st.completed == srv->st.submitted) return BSRHT_OK;
    lk.unlock();
    std::this_thread::sleep_for(std::chrono::duration<double>(kPollSleep));
    lk.lock();
  }
}

int bsrht_server_stats(bsrht_server_t srv, bsrht_server_stats_t *out) {
  if (!srv || !out) return BSRHT_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->st;
  out->queued = (int64_t)srv->queue.size();
  return BSRHT_OK;
}

int bsrht_server_set_batching(bsrht_server_t srv, int on) {
  if (!srv) return BSRHT_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->batching = on != 0;
  return BSRHT_OK;
}

double bsrht_server_clock(bsrht_server_t srv) { return srv ? srv->now() : 0.0; }

int bsrht_server_destroy(bsrht_server_t srv) {
  if (!srv) return BSRHT_EINVAL;
  bsrht_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  for (auto &t : srv->threads) t.join();
  for (auto &kv : srv->plans) {
    if (kv.second->plan) bsrht_plan_destroy(kv.second->plan);
    delete kv.second;
  }
  srv->plans.clear();
  srv->release_device();
  delete srv;
  return BSRHT_OK;
}

}  // extern "C"
