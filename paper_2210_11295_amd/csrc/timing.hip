// Instrumentation: HIP events recorded around the launches of one chosen
// kernel, on the stream that kernel runs on, so a benchmark can report that
// kernel's own duration next to the whole call's.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "common.h"

namespace bsrht {
namespace {

struct TimingState {
  int which = 0;  // BSRHT_TIMING_* of the kernel being timed, 0 = off
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t used = 0;
};

TimingState g_timing;

}  // namespace

void debug_report(const char *file, int line, const char *what, int status) {
  static const bool on = getenv("BSRHT_DEBUG") != nullptr;
  if (!on) return;
  fprintf(stderr, "[bsrht] %s:%d: %s -> status %d (%s)\n", file, line, what, status,
          bsrht_strerror(status));
}

hipEvent_t timing_begin(int which, hipStream_t s) {
  if (g_timing.which != which) return nullptr;
  if (g_timing.used == g_timing.events.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return nullptr;
    }
    g_timing.events.emplace_back(a, b);
  }
  hipEvent_t ev = g_timing.events[g_timing.used].first;
  if (hipEventRecord(ev, s) != hipSuccess) return nullptr;
  return ev;
}

void timing_end(hipEvent_t began, hipStream_t s) {
  if (!began) return;
  if (hipEventRecord(g_timing.events[g_timing.used].second, s) == hipSuccess) ++g_timing.used;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

int bsrht_timing_enable(int which) {
  g_timing.which = which;
  g_timing.used = 0;
  return BSRHT_OK;
}

int bsrht_timing_read(double *total_ms, int64_t *launches) {
  double sum = 0.0;
  for (size_t i = 0; i < g_timing.used; ++i) {
    if (hipEventSynchronize(g_timing.events[i].second) != hipSuccess) return BSRHT_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_timing.events[i].first, g_timing.events[i].second) !=
        hipSuccess)
      return BSRHT_EDEVICE;
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = (int64_t)g_timing.used;
  return BSRHT_OK;
}

}  // extern "C"
