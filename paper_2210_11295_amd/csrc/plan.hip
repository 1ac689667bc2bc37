// Plan construction: the random tables of the block SRHT (section 2,
// eq. (2.3)) built on the device from the counter-based generator, plus the
// library's small C entry points (version, error strings, plan queries).
#include <stdlib.h>
#include <string.h>

#include <new>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "philox.h"

namespace bsrht {

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

// D sign bits: one thread per 32-bit word of the bitmask over the padded
// block layout (bit g = i*rp + x for block i, position x < rp; rp = 2^log2r;
// positions x >= r of a padded block multiply zeros).  Block i, position x
// uses bit x%256 of
// philox((x/256, i, tag D, 0)).  For r >= 32 a word lies inside one block and
// one 256-bit output, so one generator call serves the whole word.
__global__ void build_d_kernel(uint32_t *Dbits, int64_t words, int64_t n,
                               int log2r, uint64_t seed) {
  int64_t wd = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (wd >= words) return;
  const int64_t r = int64_t(1) << log2r;
  const int64_t g0 = wd * 32;
  uint32_t word = 0;
  if (r >= 32) {
    const int64_t i = g0 >> log2r;
    const int64_t x = g0 & (r - 1);
    Philox4 o = philox4x64_10((uint64_t)(x >> 8), (uint64_t)i, kTagD, 0, seed, 0);
    word = philox_word32(o, (uint32_t)(x & 255));
    const int64_t valid = n - g0;
    if (valid < 32) word &= (1u << valid) - 1u;
  } else {
    for (int b = 0; b < 32; ++b) {
      const int64_t g = g0 + b;
      if (g >= n) break;
      const int64_t i = g >> log2r;
      const int64_t x = g & (r - 1);
      Philox4 o = philox4x64_10((uint64_t)(x >> 8), (uint64_t)i, kTagD, 0, seed, 0);
      word |= philox_bit(o, (uint32_t)(x & 255)) << b;
    }
  }
  Dbits[wd] = word;
}

// Dt sign bits: one thread per word (block i, word wj); bits j = 32*wj + b.
__global__ void build_dt_kernel(uint32_t *Dtbits, int64_t p, int64_t dt_words,
                                int64_t l, uint64_t seed) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p * dt_words) return;
  const int64_t i = t / dt_words;
  const int64_t wj = t - i * dt_words;
  const int64_t j0 = wj * 32;
  Philox4 o = philox4x64_10((uint64_t)(j0 >> 8), (uint64_t)i, kTagDt, 0, seed, 0);
  uint32_t word = philox_word32(o, (uint32_t)(j0 & 255));
  const int64_t valid = l - j0;
  if (valid < 32) word &= (1u << valid) - 1u;
  Dtbits[t] = word;
}

// R with replacement: R_j = word0(philox((j, 0, tag R, 0))) mod r.
__global__ void build_r_kernel(int32_t *R, int64_t l, int64_t r, uint64_t seed) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= l) return;
  Philox4 o = philox4x64_10((uint64_t)j, 0, kTagR, 0, seed, 0);
  R[j] = (int32_t)(o.w[0] & (uint64_t)(r - 1));
}

// Gather lane orders.  In the gathers every lane reads 16-byte quads of the
// LDS data of its sample's position R_j mod b, and lanes whose samples fall
// in the same bank group (but not the same row) conflict.  Column kernels:
// rows are 17 quads apart, so the c-th quad's bank group is (R_j + c) mod 16
// and the key is R_j mod 16.  Right-side kernel: position x holds 16 quads
// swizzled by (x >> 2) mod 16, so the key is (R_j >> 2) mod 16.  Within each
// consecutive group of 1024 samples an order takes the samples round-robin
// over the key (round k takes the k-th sample, in draw order, of every key
// value that has one), so that most aligned 16-lane groups hold 16 distinct
// keys.  Sample (key v, rank k) goes to position
//   sum_u min(k, size_u) + #{u < v : size_u > k}
// of its group (size_u: samples with key u in the group), a bijection.
// Only the assignment of samples to lanes changes: each sample's sum runs in
// the same order, so the sketch is bitwise the same as in draw order.
__global__ __launch_bounds__(1024) void build_order_kernel(const int32_t *__restrict__ R,
                                                           int32_t *__restrict__ order,
                                                           int64_t l, int shift) {
  __shared__ int cnt[16][16];  // [wave][residue]: counts, then exclusive prefix
  __shared__ int size[16];
  const int64_t j0 = (int64_t)blockIdx.x * 1024;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const bool ok = j0 + t < l;
  const int rho = ok ? ((R[j0 + t] >> shift) & 15) : 16;
  int rank = 0;
  for (int v = 0; v < 16; ++v) {
    const unsigned long long msk = __ballot(rho == v);
    if (rho == v) rank = __popcll(msk & ((1ull << lane) - 1ull));
    if (lane == 0) cnt[w][v] = __popcll(msk);
  }
  __syncthreads();
  if (t < 16) {
    int sum = 0;
    for (int ww = 0; ww < 16; ++ww) {
      const int c = cnt[ww][t];
      cnt[ww][t] = sum;
      sum += c;
    }
    size[t] = sum;
  }
  __syncthreads();
  if (ok) {
    const int k = cnt[w][rho] + rank;
    int pos = 0;
    for (int v = 0; v < 16; ++v) {
      const int sv = size[v];
      pos += (k < sv ? k : sv) + ((v < rho && sv > k) ? 1 : 0);
    }
    order[j0 + pos] = (int32_t)(j0 + t);
  }
}

// Rows per block padded to a power of two (section 2's partial SRHT).
static int64_t padded_block(int64_t r) {
  int64_t rp = 1;
  while (rp < r) rp <<= 1;
  return rp;
}

static bool valid_sizes(int64_t n, int64_t p, int64_t l) {
  if (n < 1 || p < 1 || l < 1 || n >= (int64_t(1) << 31)) return false;
  if (n % p) return false;
  if (p * padded_block(n / p) >= (int64_t(1) << 31)) return false;
  if (l > n) return false;
  return true;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

const char *bsrht_version(void) { return "bsrht-gfx950 0.1"; }

const char *bsrht_strerror(int status) {
  switch (status) {
    case BSRHT_OK: return "ok";
    case BSRHT_EINVAL: return "invalid argument";
    case BSRHT_ENOMEM: return "buffer too small";
    case BSRHT_EDEVICE: return "HIP runtime error";
    case BSRHT_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

size_t bsrht_plan_bytes(int64_t n, int64_t p, int64_t l) {
  if (!valid_sizes(n, p, l)) return 0;
  Sizer sz;
  sz.take<int32_t>((size_t)l);
  sz.take<uint32_t>((size_t)((p * padded_block(n / p) + 31) / 32));
  sz.take<uint32_t>((size_t)(p * ((l + 31) / 32)));
  sz.take<int32_t>((size_t)l);
  sz.take<int32_t>((size_t)l);
  return align256(sz.used);
}

int bsrht_plan(int64_t n, int64_t p, int64_t l, uint64_t seed, int sampling,
               int precision, void *dev_mem, size_t dev_bytes, void *stream,
               bsrht_plan_t *out) {
  if (!out) return BSRHT_EINVAL;
  *out = nullptr;
  if (!valid_sizes(n, p, l)) return BSRHT_EINVAL;
  if (sampling != BSRHT_WITH_REPLACEMENT && sampling != BSRHT_WITHOUT_REPLACEMENT)
    return BSRHT_EINVAL;
  if (precision != BSRHT_FP32 && precision != BSRHT_SPLIT_BF16) return BSRHT_EINVAL;
  const int64_t r = n / p, rp = padded_block(r);
  if (sampling == BSRHT_WITHOUT_REPLACEMENT && l > rp) return BSRHT_EINVAL;
  if (!dev_mem) return BSRHT_EINVAL;
  if (dev_bytes < bsrht_plan_bytes(n, p, l)) return BSRHT_ENOMEM;

  bsrht_plan_s *pl = new (std::nothrow) bsrht_plan_s;
  if (!pl) return BSRHT_ENOMEM;
  pl->n = n;
  pl->p = p;
  pl->l = l;
  pl->r = r;
  pl->rp = rp;
  pl->log2r = ilog2_i64(rp);
  pl->seed = seed;
  pl->sampling = sampling;
  pl->precision = precision;
  pl->d_words = (p * rp + 31) / 32;
  pl->dt_words = (l + 31) / 32;
  pl->stream = (hipStream_t)stream;
  if (hipGetDevice(&pl->device) != hipSuccess) {
    delete pl;
    return BSRHT_EDEVICE;
  }
  Carve cv(dev_mem, dev_bytes);
  pl->R = cv.take<int32_t>((size_t)l);
  pl->Dbits = cv.take<uint32_t>((size_t)pl->d_words);
  pl->Dtbits = cv.take<uint32_t>((size_t)(p * pl->dt_words));
  pl->order = cv.take<int32_t>((size_t)l);
  pl->order_right = cv.take<int32_t>((size_t)l);
  hipStream_t s = pl->stream;

  const int tb = 256;
  build_d_kernel<<<(unsigned)((pl->d_words + tb - 1) / tb), tb, 0, s>>>(
      pl->Dbits, pl->d_words, p * rp, pl->log2r, seed);
  build_dt_kernel<<<(unsigned)((p * pl->dt_words + tb - 1) / tb), tb, 0, s>>>(
      pl->Dtbits, p, pl->dt_words, l, seed);
  if (sampling == BSRHT_WITH_REPLACEMENT) {
    build_r_kernel<<<(unsigned)((l + tb - 1) / tb), tb, 0, s>>>(pl->R, l, rp, seed);
  } else {
    // Partial Fisher-Yates is sequential in j; it runs on the host with the
    // same generator and is uploaded once.  A sparse pool keeps it O(l).
    std::vector<int32_t> Rh((size_t)l);
    std::unordered_map<int64_t, int64_t> pool;  // slots moved from identity
    auto get = [&](int64_t slot) -> int64_t {
      auto it = pool.find(slot);
      return it == pool.end() ? slot : it->second;
    };
    for (int64_t j = 0; j < l; ++j) {
      Philox4 o = philox4x64_10((uint64_t)j, 0, kTagR, 0, seed, 0);
      uint64_t hi, lo;
      mul_hilo64(o.w[0], (uint64_t)(rp - j), hi, lo);
      const int64_t t = j + (int64_t)hi;
      const int64_t pj = get(j), pt = get(t);
      pool[j] = pt;
      pool[t] = pj;
      Rh[(size_t)j] = (int32_t)pt;
    }
    if (hipMemcpyAsync(pl->R, Rh.data(), sizeof(int32_t) * (size_t)l,
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      delete pl;
      return BSRHT_EDEVICE;
    }
  }
  build_order_kernel<<<(unsigned)((l + 1023) / 1024), 1024, 0, s>>>(pl->R, pl->order, l, 0);
  build_order_kernel<<<(unsigned)((l + 1023) / 1024), 1024, 0, s>>>(pl->R, pl->order_right, l,
                                                                    2);
  if (hipGetLastError() != hipSuccess) {
    delete pl;
    return BSRHT_EDEVICE;
  }
  *out = pl;
  return BSRHT_OK;
}

int bsrht_plan_destroy(bsrht_plan_t plan) {
  delete plan;
  return BSRHT_OK;
}

int bsrht_plan_info(bsrht_plan_t plan, int64_t *n, int64_t *p, int64_t *l,
                    int *sampling, int *precision) {
  if (!plan) return BSRHT_EINVAL;
  if (n) *n = plan->n;
  if (p) *p = plan->p;
  if (l) *l = plan->l;
  if (sampling) *sampling = plan->sampling;
  if (precision) *precision = plan->precision;
  return BSRHT_OK;
}

int bsrht_plan_export(bsrht_plan_t plan, int32_t *R, uint32_t *Dbits,
                      uint32_t *Dtbits) {
  if (!plan) return BSRHT_EINVAL;
  hipStream_t s = plan->stream;
  if (R && copy_to_host(R, plan->R, sizeof(int32_t) * (size_t)plan->l, s) != BSRHT_OK)
    return BSRHT_EDEVICE;
  if (Dbits &&
      copy_to_host(Dbits, plan->Dbits, sizeof(uint32_t) * (size_t)plan->d_words, s) != BSRHT_OK)
    return BSRHT_EDEVICE;
  if (Dtbits && copy_to_host(Dtbits, plan->Dtbits,
                             sizeof(uint32_t) * (size_t)(plan->p * plan->dt_words),
                             s) != BSRHT_OK)
    return BSRHT_EDEVICE;
  return BSRHT_OK;
}

}  // extern "C"
