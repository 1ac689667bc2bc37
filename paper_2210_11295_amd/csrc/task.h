// Stream-ordered device work as C++20 coroutines.
//
// A driver step that needs a value from the device (a Cholesky flag, a sweep
// counter, eigenvalues) awaits a readback.  With a blocking context the
// await copies and synchronises the stream on the spot, so the coroutine runs
// to completion in one call: that is how the public C entry points run.  With
// an asynchronous context the await queues the copy into pinned staging,
// records the context's event and suspends; an executor resumes the job when
// the event has completed.  One host thread can so keep several jobs in
// flight on several streams without blocking on any of them.
#pragma once

#include <coroutine>
#include <cstring>

#include "common.h"

namespace bsrht {

struct DevCtx {
  hipStream_t s = nullptr;
  bool blocking = true;
  hipEvent_t ev = nullptr;        // async: recorded at every suspension point
  char *pinned = nullptr;         // async: staging, two halves of half_bytes
  size_t half_bytes = 0;          //   (first: device -> host, second: host -> device)
  std::coroutine_handle<> resume_point;  // async: innermost suspended coroutine
};

// A coroutine returning a BSRHT_* status.  Awaiting a Task runs it as a
// sub-step of the awaiting coroutine (it resumes its parent when it ends).
class Task {
 public:
  struct promise_type {
    int status = BSRHT_OK;
    std::coroutine_handle<> parent;
    Task get_return_object() {
      return Task(std::coroutine_handle<promise_type>::from_promise(*this));
    }
    std::suspend_always initial_suspend() noexcept { return {}; }
    struct Final {
      bool await_ready() noexcept { return false; }
      std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
        auto p = h.promise().parent;
        return p ? p : std::noop_coroutine();
      }
      void await_resume() noexcept {}
    };
    Final final_suspend() noexcept { return {}; }
    void return_value(int st) { status = st; }
    void unhandled_exception() { std::terminate(); }
  };

  explicit Task(std::coroutine_handle<promise_type> h) : h_(h) {}
  Task(Task &&o) noexcept : h_(o.h_) { o.h_ = {}; }
  Task &operator=(Task &&o) noexcept {
    if (this != &o) {
      if (h_) h_.destroy();
      h_ = o.h_;
      o.h_ = {};
    }
    return *this;
  }
  Task(const Task &) = delete;
  Task &operator=(const Task &) = delete;
  ~Task() {
    if (h_) h_.destroy();
  }

  bool done() const { return !h_ || h_.done(); }
  int status() const { return h_ ? h_.promise().status : BSRHT_EINVAL; }
  void start() { h_.resume(); }

  // as a sub-step
  bool await_ready() const noexcept { return false; }
  std::coroutine_handle<> await_suspend(std::coroutine_handle<> parent) noexcept {
    h_.promise().parent = parent;
    return h_;
  }
  int await_resume() const noexcept { return h_.promise().status; }

 private:
  std::coroutine_handle<promise_type> h_;
};

// Runs a task to completion with a blocking context.
inline int run_blocking(Task t) {
  t.start();
  return t.done() ? t.status() : BSRHT_EDEVICE;
}

// co_await readback(ctx, dst, src, bytes): host dst <- device src after all
// work queued so far on ctx.s.  Yields a BSRHT_* status.
struct Readback {
  DevCtx &ctx;
  void *dst;
  const void *src;
  size_t bytes;
  int st = BSRHT_OK;
  bool await_ready() {
    if (ctx.blocking || bytes > ctx.half_bytes) {
      st = copy_to_host(dst, src, bytes, ctx.s);
      return true;
    }
    if (hipMemcpyAsync(ctx.pinned, src, bytes, hipMemcpyDeviceToHost, ctx.s) != hipSuccess ||
        hipEventRecord(ctx.ev, ctx.s) != hipSuccess) {
      st = BSRHT_EDEVICE;
      return true;
    }
    return false;
  }
  void await_suspend(std::coroutine_handle<> h) { ctx.resume_point = h; }
  int await_resume() {
    if (!ctx.blocking && bytes <= ctx.half_bytes && st == BSRHT_OK)
      std::memcpy(dst, ctx.pinned, bytes);
    return st;
  }
};
inline Readback readback(DevCtx &ctx, void *dst, const void *src, size_t bytes) {
  return Readback{ctx, dst, src, bytes};
}

// co_await upload(ctx, dst, src, bytes): device dst <- host src, ordered on
// ctx.s; the host buffer may be reused once the await has returned.
struct Upload {
  DevCtx &ctx;
  void *dst;
  const void *src;
  size_t bytes;
  int st = BSRHT_OK;
  bool await_ready() {
    if (ctx.blocking || bytes > ctx.half_bytes) {
      st = copy_to_device(dst, src, bytes, ctx.s);
      return true;
    }
    char *stage = ctx.pinned + ctx.half_bytes;
    std::memcpy(stage, src, bytes);
    if (hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, ctx.s) != hipSuccess ||
        hipEventRecord(ctx.ev, ctx.s) != hipSuccess) {
      st = BSRHT_EDEVICE;
      return true;
    }
    return false;  // resume once the staging has been consumed
  }
  void await_suspend(std::coroutine_handle<> h) { ctx.resume_point = h; }
  int await_resume() { return st; }
};
inline Upload upload(DevCtx &ctx, void *dst, const void *src, size_t bytes) {
  return Upload{ctx, dst, src, bytes};
}

// co_await drained(ctx): all work queued so far on ctx.s has finished.
struct Drained {
  DevCtx &ctx;
  int st = BSRHT_OK;
  bool await_ready() {
    if (ctx.blocking) {
      st = hipStreamSynchronize(ctx.s) == hipSuccess ? BSRHT_OK : BSRHT_EDEVICE;
      return true;
    }
    if (hipEventRecord(ctx.ev, ctx.s) != hipSuccess) {
      st = BSRHT_EDEVICE;
      return true;
    }
    return false;
  }
  void await_suspend(std::coroutine_handle<> h) { ctx.resume_point = h; }
  int await_resume() { return st; }
};
inline Drained drained(DevCtx &ctx) { return Drained{ctx}; }

#define BSRHT_CO_LAUNCH_CHECK()                                                  \
  do {                                                                           \
    if (hipGetLastError() != hipSuccess) {                                       \
      ::bsrht::debug_report(__FILE__, __LINE__, "kernel launch", BSRHT_EDEVICE); \
      co_return BSRHT_EDEVICE;                                                   \
    }                                                                            \
  } while (0)

#define BSRHT_CO_TRY(expr)                                       \
  do {                                                           \
    const int st_ = (expr);                                      \
    if (st_ != BSRHT_OK) {                                       \
      ::bsrht::debug_report(__FILE__, __LINE__, #expr, st_);     \
      co_return st_;                                             \
    }                                                            \
  } while (0)

// Job coroutines of the drivers (argument checks are the caller's).
Task rsvd_task(DevCtx &ctx, const bsrht_plan_s *plan, const float *A, int64_t m, int64_t lda,
               int64_t k, float *U, double *S, float *V, int32_t *info, void *ws,
               size_t ws_bytes);
Task nystrom_task(DevCtx &ctx, const bsrht_plan_s *plan, const float *A, int64_t lda, int64_t k,
                  float *U, double *lambda, int32_t *info, void *ws, size_t ws_bytes,
                  bool shifted);
Task jacobi_svd_task(DevCtx &ctx, double *X, int64_t nr, int64_t nc, int64_t ldx, double *V,
                     double *S, double *Us, int64_t ldu, int32_t *perm, unsigned int *flags,
                     int max_sweeps, int32_t *info, int form);

}  // namespace bsrht
