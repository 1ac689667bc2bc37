// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bsrht.h"

struct bsrht_plan_s {
  int64_t n, p, l, r;  // r = n/p rows per block
  int64_t rp;          // 2^log2r >= r: a block is padded with zeros to rp rows
  int log2r;
  uint64_t seed;
  int sampling, precision;
  int32_t *R;         // device, l entries in [0, rp), draw order
  uint32_t *Dbits;    // device, ceil(p*rp/32) words; bit i*rp + x = sign of D^(i)_x
  uint32_t *Dtbits;   // device, p * dt_words words; block i at i*dt_words
  int32_t *order;     // device, l entries: the sample served by each gather lane
                      // of the column kernels (a permutation of 0..l-1)
  int32_t *order_right;  // device, l entries: the same for the right-side kernel
  int64_t d_words, dt_words;
  hipStream_t stream; // stream the tables were written on
  int device;
};

namespace bsrht {

// With BSRHT_DEBUG set in the environment, failures print where they
// happened (stderr); otherwise they only return the status.
void debug_report(const char *file, int line, const char *what, int status);

#define BSRHT_HIP_CHECK(expr)                                        \
  do {                                                               \
    if ((expr) != hipSuccess) {                                      \
      ::bsrht::debug_report(__FILE__, __LINE__, #expr, BSRHT_EDEVICE); \
      return BSRHT_EDEVICE;                                          \
    }                                                                \
  } while (0)

#define BSRHT_LAUNCH_CHECK()                                                     \
  do {                                                                           \
    if (hipGetLastError() != hipSuccess) {                                       \
      ::bsrht::debug_report(__FILE__, __LINE__, "kernel launch", BSRHT_EDEVICE); \
      return BSRHT_EDEVICE;                                                      \
    }                                                                            \
  } while (0)

// Propagate a non-OK status from a library call, with the debug trace.
#define BSRHT_TRY(expr)                                          \
  do {                                                           \
    const int st_ = (expr);                                      \
    if (st_ != BSRHT_OK) {                                       \
      ::bsrht::debug_report(__FILE__, __LINE__, #expr, st_);     \
      return st_;                                                \
    }                                                            \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Work items one launch dimension can dispatch (grid size x workgroup size
// must fit in 32 bits), less one workgroup of slack.
constexpr int64_t kMaxGridItems = int64_t(0xFFFFFFFF) - 1024;

// Workgroups of tb threads for a grid-stride loop over `total` items: one
// per tb items, at most 65536 (each thread then takes several items).
inline unsigned stride_grid(int64_t total, int tb) {
  const int64_t g = (total + tb - 1) / tb;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

inline int ilog2_i64(int64_t x) {
  int k = 0;
  while ((int64_t(1) << k) < x) ++k;
  return k;
}

// Number of compute units of the current device (256 on MI355X).
int device_cu_count();

// Workspace carving: successive 256-byte aligned regions of a caller buffer.
struct Carve {
  char *base;
  size_t size;
  size_t used = 0;
  bool overflow = false;
  Carve(void *b, size_t s) : base(static_cast<char *>(b)), size(s) {}
  template <class T>
  T *take(size_t count) {
    size_t off = align256(used);
    size_t bytes = count * sizeof(T);
    used = off + bytes;
    if (used > size || (base == nullptr && bytes > 0)) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T *>(base + off);
  }
};

// Workspace sizing mirrors Carve exactly.
struct Sizer {
  size_t used = 0;
  template <class T>
  void take(size_t count) { used = align256(used) + count * sizeof(T); }
};

// The sketch Y = Omega A for row-major A (n x m, lda) into Y (l x m, ldy).
// ws must hold apply_ws_bytes(plan, m).  Used by bsrht_apply and by the
// RSVD / Nystrom drivers.
size_t apply_ws_bytes(const bsrht_plan_s *plan, int64_t m);
int apply_fp32(const bsrht_plan_s *plan, const float *A, int64_t m, int64_t lda,
               float *Y, int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s);
int apply_split_bf16(const bsrht_plan_s *plan, const float *A, int64_t m,
                     int64_t lda, float *Y, int64_t ldy, void *ws,
                     size_t ws_bytes, hipStream_t s);
size_t apply_split_bf16_ws_bytes(const bsrht_plan_s *plan, int64_t m);
size_t apply_fp32_ws_bytes(const bsrht_plan_s *plan, int64_t m);
// Y = A Omega^T for row-major A (m x n, lda) into Y (m x l, ldy); ws must
// hold apply_right_ws_bytes(plan, m).
size_t apply_right_ws_bytes(const bsrht_plan_s *plan, int64_t m);
int apply_right_fp32(const bsrht_plan_s *plan, const float *A, int64_t m, int64_t lda,
                     float *Y, int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s);
// Y[j][c] = scale * sum_s part[s][j][c] over the splits in ascending order.
int reduce_splits(const float *part, int splits, int64_t split_stride, int64_t l, int64_t m,
                  float *Y, int64_t ldy, float scale, hipStream_t s);

// Blocking copies ordered on stream s: the copy is queued on s and s is then
// synchronised, so concurrent callers on other streams are never serialised
// through the null stream.  Host memory may be pageable.
int copy_to_host(void *dst, const void *src, size_t bytes, hipStream_t s);
int copy_to_device(void *dst, const void *src, size_t bytes, hipStream_t s);

// Instrumentation hooks around the launch of the kernel selected by
// bsrht_timing_enable (no-ops otherwise).  Thread-safe.
int timing_begin(int which, hipStream_t s);  // slot handle, -1 when not timing
void timing_end(int slot, hipStream_t s);

// Release of the library's process-lifetime HIP objects (bsrht_finalize):
// the timing events, and the batched launch's graphs with their pinned
// staging and events (every table, or one table on the current device).
void release_timing_events();
int release_batch_graphs(const void *table, bool all);

}  // namespace bsrht
