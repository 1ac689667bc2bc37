// Instrumentation: HIP events recorded around the launches of one chosen
// kernel, on the stream that kernel runs on, so a benchmark can report that
// kernel's own duration next to the whole call's.
#include <stdio.h>
#include <stdlib.h>

#include <mutex>
#include <vector>

#include "common.h"

namespace bsrht {
namespace {

struct TimingState {
  int which = 0;  // BSRHT_TIMING_* of the kernel being timed, 0 = off
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  std::vector<char> done;  // the slot's end event was recorded
  size_t used = 0;         // slots handed out since timing_enable
};

TimingState g_timing;
std::mutex g_timing_mu;

}  // namespace

int copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return BSRHT_OK;
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return BSRHT_EDEVICE;
  return BSRHT_OK;
}

int copy_to_device(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return BSRHT_OK;
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return BSRHT_EDEVICE;
  return BSRHT_OK;
}

void debug_report(const char *file, int line, const char *what, int status) {
  static const bool on = getenv("BSRHT_DEBUG") != nullptr;
  if (!on) return;
  fprintf(stderr, "[bsrht] %s:%d: %s -> status %d (%s)\n", file, line, what, status,
          bsrht_strerror(status));
}

int timing_begin(int which, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (g_timing.which == 0 || g_timing.which != which) return -1;
  if (g_timing.used == g_timing.events.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    g_timing.events.emplace_back(a, b);
    g_timing.done.push_back(0);
  }
  const int slot = (int)g_timing.used;
  if (hipEventRecord(g_timing.events[(size_t)slot].first, s) != hipSuccess) return -1;
  g_timing.done[(size_t)slot] = 0;
  ++g_timing.used;
  return slot;
}

void timing_end(int slot, hipStream_t s) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if ((size_t)slot >= g_timing.used) return;  // timing was re-enabled meanwhile
  if (hipEventRecord(g_timing.events[(size_t)slot].second, s) == hipSuccess)
    g_timing.done[(size_t)slot] = 1;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

int bsrht_timing_enable(int which) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing.which = which;
  g_timing.used = 0;
  return BSRHT_OK;
}

int bsrht_timing_read(double *total_ms, int64_t *launches) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  double sum = 0.0;
  int64_t count = 0;
  for (size_t i = 0; i < g_timing.used; ++i) {
    if (!g_timing.done[i]) continue;
    if (hipEventSynchronize(g_timing.events[i].second) != hipSuccess) return BSRHT_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_timing.events[i].first, g_timing.events[i].second) !=
        hipSuccess)
      return BSRHT_EDEVICE;
    sum += ms;
    ++count;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = count;
  return BSRHT_OK;
}

}  // extern "C"
