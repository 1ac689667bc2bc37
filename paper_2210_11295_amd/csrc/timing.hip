// Instrumentation: HIP events recorded around the launches of one chosen
// kernel, on the stream that kernel runs on, so a benchmark can report that
// kernel's own duration next to the whole call's; and a plain read kernel
// that measures the HBM read rate the sketch kernels are compared with.
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

constexpr int kStreamThreads = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Reads x[0 .. n4) once (16-byte non-temporal loads, eight in flight per
// thread, grid-stride so that the whole grid sweeps one contiguous region at
// a time) and writes one partial sum per workgroup, which keeps the loads
// live.  The sums are not part of any result.
__global__ __launch_bounds__(kStreamThreads) void stream_read_kernel(const f32x4 *__restrict__ x,
                                                                     int64_t n4,
                                                                     float *__restrict__ out) {
  __shared__ float red[kStreamThreads];
  const int64_t stride = (int64_t)gridDim.x * kStreamThreads;
  int64_t i = (int64_t)blockIdx.x * kStreamThreads + threadIdx.x;
  float acc = 0.f;
  for (; i + 7 * stride < n4; i += 8 * stride) {
    f32x4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(x + i + u * stride);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n4; i += stride) {
    const f32x4 v = __builtin_nontemporal_load(x + i);
    acc += (v.x + v.y) + (v.z + v.w);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kStreamThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

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

void release_timing_events() {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto &e : g_timing.events) {
    (void)hipEventSynchronize(e.second);
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g_timing.events.clear();
  g_timing.done.clear();
  g_timing.used = 0;
  g_timing.which = 0;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

int bsrht_finalize(void) {
  release_timing_events();
  return release_batch_graphs(nullptr, true);
}

int bsrht_timing_enable(int which) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing.which = which;
  g_timing.used = 0;
  return BSRHT_OK;
}

int bsrht_timing_samples(float *ms, int64_t cap, int64_t *count) {
  if (cap < 0 || (cap > 0 && !ms)) return BSRHT_EINVAL;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  int64_t k = 0;
  for (size_t i = 0; i < g_timing.used; ++i) {
    if (!g_timing.done[i]) continue;
    if (hipEventSynchronize(g_timing.events[i].second) != hipSuccess) return BSRHT_EDEVICE;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_timing.events[i].first, g_timing.events[i].second) !=
        hipSuccess)
      return BSRHT_EDEVICE;
    if (k < cap) ms[k] = t;
    ++k;
  }
  if (count) *count = k;
  return BSRHT_OK;
}

int bsrht_stream_read(const float *x, int64_t count, float *out, void *stream) {
  if (!x || !out || count < 0 || ((uintptr_t)x & 15) != 0) return BSRHT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int slot = timing_begin(BSRHT_TIMING_STREAM, s);
  stream_read_kernel<<<BSRHT_STREAM_BLOCKS, kStreamThreads, 0, s>>>(
      reinterpret_cast<const f32x4 *>(x), count / 4, out);
  timing_end(slot, s);
  return hipGetLastError() == hipSuccess ? BSRHT_OK : BSRHT_EDEVICE;
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
