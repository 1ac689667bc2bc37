// Dense sketches Y = G A with a Gaussian or Rademacher G (l x n): the
// embeddings the block SRHT is compared with in section 4.  G is drawn from
// the same counter-based Philox4x64-10 as the block SRHT tables, key
// (seed, 0), so any entry can be generated independently:
//   Gaussian   G[j][x] = z / sqrt(l): counter (x >> 3, j, 4, 0); word
//              q = (x & 7) >> 1 gives u1 = (lo + 1/2) 2^-32 from its low and
//              u2 = (hi + 1/2) 2^-32 from its high 32 bits, rho =
//              sqrt(-2 ln u1), and z = rho cos(2 pi u2) for even x,
//              rho sin(2 pi u2) for odd x (Box-Muller; evaluated in FP64 and
//              rounded once to FP32);
//   Rademacher G[j][x] = +-1 / sqrt(l): bit (x & 255) of philox((x >> 8, j, 5,
//              0)), bit 1 -> -1.
// G is written to the workspace (l x n FP32, rows padded to 4 elements) by a
// generation kernel, then Y = G A runs on the FP32 matrix cores with the K = n
// range split into FP64 partials summed in fixed order.  This is the dense
// product the block SRHT avoids: 2 l m n flops against ~n m log2(b) adds.
#include <limits.h>

#include "common.h"
#include "dense.h"
#include "philox.h"

namespace bsrht {
namespace {

enum : uint64_t { kTagGauss = 4, kTagRad = 5 };

// One work item per 8 consecutive columns x0 .. x0+7 of row j; a grid-stride
// loop covers every item, so the grid stays within the dispatch limits.
__global__ void gen_gauss_kernel(float *__restrict__ G, int64_t l, int64_t n, int64_t ldg,
                                 uint64_t seed, double scale) {
  const int64_t n8 = (n + 7) >> 3;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < l * n8;
       idx += stride) {
    const int64_t j = idx / n8, x0 = (idx - j * n8) << 3;
    const Philox4 o = philox4x64_10((uint64_t)(x0 >> 3), (uint64_t)j, kTagGauss, 0, seed, 0);
    float z[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double u1 = ((double)(uint32_t)o.w[q] + 0.5) * 0x1p-32;
      const double u2 = ((double)(uint32_t)(o.w[q] >> 32) + 0.5) * 0x1p-32;
      const double rho = sqrt(-2.0 * log(u1));
      double sn, cs;
      sincospi(2.0 * u2, &sn, &cs);
      z[2 * q] = (float)(rho * cs * scale);
      z[2 * q + 1] = (float)(rho * sn * scale);
    }
    float *row = G + j * ldg + x0;
    if (x0 + 8 <= n && ((uintptr_t)row & 15) == 0) {
      reinterpret_cast<float4 *>(row)[0] = make_float4(z[0], z[1], z[2], z[3]);
      reinterpret_cast<float4 *>(row)[1] = make_float4(z[4], z[5], z[6], z[7]);
    } else {
      for (int e = 0; e < 8 && x0 + e < n; ++e) row[e] = z[e];
    }
  }
}

// One work item per 8 consecutive columns (32 neighbouring items share a
// 256-bit output); grid-stride as above.
__global__ void gen_rademacher_kernel(float *__restrict__ G, int64_t l, int64_t n, int64_t ldg,
                                      uint64_t seed, float scale) {
  const int64_t n8 = (n + 7) >> 3;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < l * n8;
       idx += stride) {
    const int64_t j = idx / n8, x0 = (idx - j * n8) << 3;
    const Philox4 o = philox4x64_10((uint64_t)(x0 >> 8), (uint64_t)j, kTagRad, 0, seed, 0);
    float *row = G + j * ldg + x0;
    for (int e = 0; e < 8 && x0 + e < n; ++e)
      row[e] = philox_bit(o, (uint32_t)((x0 + e) & 255)) ? -scale : scale;
  }
}

struct DenseLayout {
  int64_t ldg = 0;
  int splits = 1;
  size_t g_bytes = 0, part_bytes = 0;
};

DenseLayout dense_layout(int64_t n, int64_t l, int64_t m) {
  DenseLayout L;
  L.ldg = (n + 3) & ~int64_t(3);
  L.g_bytes = align256((size_t)(l * L.ldg) * sizeof(float));
  // Split the K = n range so that ~2 workgroups run per compute unit, with at
  // least 512 terms of K per split.
  const int64_t tiles = ((l + 127) / 128) * ((m + 127) / 128);
  int64_t sp = (2 * (int64_t)device_cu_count() + tiles - 1) / tiles;
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, n / 512));
  sp = std::max<int64_t>(1, std::min<int64_t>(sp, 256));
  L.splits = (int)sp;
  L.part_bytes = L.splits > 1 ? align256((size_t)(L.splits * l * m) * sizeof(double)) : 0;
  return L;
}

}  // namespace
}  // namespace bsrht

using namespace bsrht;

extern "C" {

size_t bsrht_dense_workspace(int64_t n, int64_t l, int64_t m) {
  if (n < 1 || l < 1 || m < 1) return 0;
  const DenseLayout L = dense_layout(n, l, m);
  return L.g_bytes + L.part_bytes;
}

int bsrht_dense_sketch(int kind, uint64_t seed, int64_t n, int64_t l, const float *A, int64_t m,
                       int64_t lda, float *Y, int64_t ldy, void *ws, size_t ws_bytes,
                       void *stream) {
  if ((kind != BSRHT_DENSE_GAUSSIAN && kind != BSRHT_DENSE_RADEMACHER) || n < 1 || l < 1 ||
      m < 0)
    return BSRHT_EINVAL;
  if (m == 0) return BSRHT_OK;
  if (!A || !Y || lda < m || ldy < m) return BSRHT_EINVAL;
  if (n > INT_MAX || l > INT_MAX || m > INT_MAX) return BSRHT_EUNSUPPORTED;
  const DenseLayout L = dense_layout(n, l, m);
  if (!ws || ws_bytes < L.g_bytes + L.part_bytes) return BSRHT_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  float *G = static_cast<float *>(ws);
  double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + L.g_bytes);
  const int64_t total = l * ((n + 7) >> 3);
  const unsigned blocks = stride_grid(total, 256);
  if (kind == BSRHT_DENSE_GAUSSIAN)
    gen_gauss_kernel<<<blocks, 256, 0, s>>>(G, l, n, L.ldg, seed, 1.0 / sqrt((double)l));
  else
    gen_rademacher_kernel<<<blocks, 256, 0, s>>>(G, l, n, L.ldg, seed,
                                                 (float)(1.0 / sqrt((double)l)));
  BSRHT_LAUNCH_CHECK();
  GemmDesc d;
  d.M = l; d.N = m; d.K = n;
  d.sai = L.ldg; d.sak = 1;
  d.sbk = lda; d.sbj = 1;
  d.ldc = ldy;
  const int tslot = timing_begin(BSRHT_TIMING_DENSE_GEMM, s);
  const int st = gemm_f32_splitk(d, G, A, Y, part, L.splits, s);
  timing_end(tslot, s);
  return st;
}

}  // extern "C"
