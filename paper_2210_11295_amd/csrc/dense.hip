// Dense linear-algebra kernels behind the randomized SVD (section 3.1,
// Algorithm 1) and the Nystrom approximation (section 3.2, Algorithm 2):
//   - matrix-core GEMM, C = alpha * A B (+ beta C) with strided operands,
//     FP32 (v_mfma_f32_16x16x4f32) or FP64 (v_mfma_f64_16x16x4f64), split-K;
//   - FP64 Cholesky C^T C = G (upper C), the factorisation behind
//     Cholesky-QR (used where the paper's Algorithms ask for QR / TSQR);
//   - inverse of an upper-triangular matrix;
//   - one-sided (Hestenes) block Jacobi SVD, the "SVD of R" step of both
//     Algorithms: block pairs swept in LDS, one launch per round;
//   - small helpers (identity, transpose/convert, column scaling, sort).
#include <algorithm>

#include "common.h"
#include "dense.h"
#include "task.h"

namespace bsrht {
namespace {

constexpr int kTM = 64, kTN = 64, kTK = 16;  // GEMM workgroup tile
constexpr int kGemmThreads = 256;            // 4 waves, each a 32 x 32 sub-tile

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }

// One workgroup computes a kTM x kTN tile of C over the K range of its split.
// A[i][k] = A[i*sai + k*sak], B[k][j] = B[k*sbk + j*sbj].
template <typename TA, typename TB, typename TC, bool F64>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(GemmDesc d, const TA *__restrict__ A,
                                                            const TB *__restrict__ B,
                                                            TC *__restrict__ C) {
  using TS = typename std::conditional<F64, double, float>::type;
  __shared__ TS As[kTK][kTM + 1];
  __shared__ TS Bs[kTK][kTN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kTM, j0 = (int64_t)blockIdx.y * kTN;
  const int64_t kchunk = (d.K + gridDim.z - 1) / gridDim.z;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(d.K, kb + kchunk);
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;  // wave sub-tile origin
  using Acc = typename std::conditional<F64, double __attribute__((ext_vector_type(4))),
                                        float __attribute__((ext_vector_type(4)))>::type;
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  const bool a_icontig = d.sai == 1;
  const bool b_jcontig = d.sbj == 1;
  for (int64_t k0 = kb; k0 < ke; k0 += kTK) {
    // stage A (kTM x kTK) and B (kTK x kTN), zero-filled outside the matrix
#pragma unroll
    for (int r = 0; r < (kTM * kTK) / kGemmThreads; ++r) {
      const int e = tid + r * kGemmThreads;
      int ii, kk;
      if (a_icontig) {
        ii = e % kTM;
        kk = e / kTM;
      } else {
        ii = e / kTK;
        kk = e % kTK;
      }
      const int64_t gi = i0 + ii, gk = k0 + kk;
      TS v = 0;
      if (gi < d.M && gk < ke) v = (TS)A[gi * d.sai + gk * d.sak];
      As[kk][ii] = v;
    }
#pragma unroll
    for (int r = 0; r < (kTN * kTK) / kGemmThreads; ++r) {
      const int e = tid + r * kGemmThreads;
      int jj, kk;
      if (b_jcontig) {
        jj = e % kTN;
        kk = e / kTN;
      } else {
        jj = e / kTK;
        kk = e % kTK;
      }
      const int64_t gj = j0 + jj, gk = k0 + kk;
      TS v = 0;
      if (gj < d.N && gk < ke) v = (TS)B[gk * d.sbk + gj * d.sbj];
      Bs[kk][jj] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 4) {
      const int kk = ks + (lane >> 4);
      TS a0 = As[kk][wi + (lane & 15)], a1 = As[kk][wi + 16 + (lane & 15)];
      TS b0 = Bs[kk][wj + (lane & 15)], b1 = Bs[kk][wj + 16 + (lane & 15)];
      if constexpr (F64) {
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      } else {
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // D layout of the 16x16 blocks, lane l, item v, column l%16: row
  // 4*(l/16)+v for the FP32 instruction and l/16 + 4v for the FP64 one.
  TC *Cz = C + (int64_t)blockIdx.z * d.split_stride;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + wi + 16 * a + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        const int64_t gj = j0 + wj + 16 * b + (lane & 15);
        if (gi < d.M && gj < d.N) {
          const double val = d.alpha * (double)acc[a][b][v];
          TC *dst = Cz + gi * d.ldc + gj;
          if (d.beta != 0.0)
            *dst = (TC)(val + d.beta * (double)*dst);
          else
            *dst = (TC)val;
        }
      }
}

// ---------------------------------------------------------------------------
// Large-tile GEMM for the tall products (Z = A Q, the Gram Z^T Z, U = Z M):
// a 128 x 128 workgroup tile, 4 waves of 64 x 64 (4 x 4 MFMA blocks each),
// 16-wide k tiles double-buffered in LDS with one barrier per tile and the
// next tile's 16-byte global loads in flight during the MFMAs.  Used when B
// is j-contiguous and A is k-contiguous (AK) or i-contiguous (!AK), with
// 16-byte aligned bases and strides that are multiples of 4 elements; the
// split-K chunks are multiples of the k tile.  Other shapes take gemm_kernel.
constexpr int kBM = 128, kBN = 128, kBK = 16, kBPad = 4;
constexpr int kBThreads = 256;

template <typename T>
struct Vec4 {
  T v[4];
};

// Four consecutive elements at p (16-byte aligned for float, 32 for double).
template <typename T>
__device__ __forceinline__ Vec4<T> load4(const T *p) {
  Vec4<T> r;
  if constexpr (sizeof(T) == 4) {
    const float4 f = *reinterpret_cast<const float4 *>(p);
    r.v[0] = f.x;
    r.v[1] = f.y;
    r.v[2] = f.z;
    r.v[3] = f.w;
  } else {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    r.v[0] = a.x;
    r.v[1] = a.y;
    r.v[2] = b.x;
    r.v[3] = b.y;
  }
  return r;
}

template <typename TA, typename TB, typename TC, bool F64, bool AK>
__global__ __launch_bounds__(kBThreads) void gemm_big_kernel(GemmDesc d, const TA *__restrict__ A,
                                                             const TB *__restrict__ B,
                                                             TC *__restrict__ C) {
  using TS = typename std::conditional<F64, double, float>::type;
  constexpr int KT = kBK;
  constexpr int NV = KT / 8;  // 4-element vectors per thread per operand and tile
  __shared__ __attribute__((aligned(16))) TS As[2][KT][kBM + kBPad];
  __shared__ __attribute__((aligned(16))) TS Bs[2][KT][kBN + kBPad];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  if (d.upper_tiles && blockIdx.x > blockIdx.y) return;  // mirrored by the caller
  const int64_t i0 = (int64_t)blockIdx.x * kBM, j0 = (int64_t)blockIdx.y * kBN;
  int64_t kchunk = (d.K + gridDim.z - 1) / gridDim.z;
  kchunk = (kchunk + KT - 1) / KT * KT;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(d.K, kb + kchunk);
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  const bool ij_inside = i0 + kBM <= d.M && j0 + kBN <= d.N;
  using Acc = typename std::conditional<F64, double __attribute__((ext_vector_type(4))),
                                        float __attribute__((ext_vector_type(4)))>::type;
  Acc acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  // Each thread moves NV 4-element vectors of A and NV of B per k tile.  They
  // stay in the storage type until staged: a conversion right after the load
  // would make the load wait at once instead of overlapping the MFMAs.
  Vec4<TA> ra[NV];
  Vec4<TB> rb[NV];
  auto a_pos = [&](int v, int64_t k0, int64_t &gi, int64_t &gk) {
    if constexpr (AK) {  // 128 rows x KT/4 vectors of k
      gi = i0 + v / (KT / 4);
      gk = k0 + 4 * (v % (KT / 4));
    } else {             // KT k rows x 32 vectors of i
      gk = k0 + (v >> 5);
      gi = i0 + 4 * (v & 31);
    }
  };
  auto fetch = [&](int64_t k0) {
    if (ij_inside && k0 + KT <= ke) {  // whole tile in range (uniform branch)
#pragma unroll
      for (int h = 0; h < NV; ++h) {
        const int v = tid + h * kBThreads;
        int64_t gi, gk;
        a_pos(v, k0, gi, gk);
        ra[h] = load4<TA>(A + gi * d.sai + gk * d.sak);
        rb[h] = load4<TB>(B + (k0 + (v >> 5)) * d.sbk + j0 + 4 * (v & 31));
      }
      return;
    }
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const int v = tid + h * kBThreads;
      int64_t gi, gk;
      a_pos(v, k0, gi, gk);
      const TA *src = A + gi * d.sai + gk * d.sak;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool in = AK ? (gi < d.M && gk + e < ke) : (gk < ke && gi + e < d.M);
        ra[h].v[e] = in ? src[AK ? e : e * d.sai] : (TA)0;
      }
      // B: KT k rows x 32 vectors of j
      const int64_t bk = k0 + (v >> 5), bj = j0 + 4 * (v & 31);
      const TB *bsrc = B + bk * d.sbk + bj;
#pragma unroll
      for (int e = 0; e < 4; ++e) rb[h].v[e] = (bk < ke && bj + e < d.N) ? bsrc[e] : (TB)0;
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int h = 0; h < NV; ++h) {
      const int v = tid + h * kBThreads;
      if constexpr (AK) {
        const int ii = v / (KT / 4), kk = 4 * (v % (KT / 4));
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][kk + e][ii] = (TS)ra[h].v[e];
      } else {
        const int kk = v >> 5, ii = 4 * (v & 31);
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][kk][ii + e] = (TS)ra[h].v[e];
      }
      const int kk = v >> 5, jj = 4 * (v & 31);
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[buf][kk][jj + e] = (TS)rb[h].v[e];
    }
  };

  const int64_t ntiles = (ke - kb + KT - 1) / KT;
  if (ntiles > 0) {
    fetch(kb);
    stage(0);
  }
  __syncthreads();
  for (int64_t t = 0; t < ntiles; ++t) {
    const int cur = (int)(t & 1);
    const bool more = t + 1 < ntiles;
    if (more) fetch(kb + (t + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT; ks += 4) {
      const int kk = ks + (lane >> 4);
      TS av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[cur][kk][wi + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[cur][kk][wj + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (F64)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    if (more) stage(cur ^ 1);
    __syncthreads();
  }
  TC *Cz = C + (int64_t)blockIdx.z * d.split_stride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + wi + 16 * a + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        const int64_t gj = j0 + wj + 16 * b + (lane & 15);
        if (gi < d.M && gj < d.N) {
          const double val = d.alpha * (double)acc[a][b][v];
          TC *dst = Cz + gi * d.ldc + gj;
          if (d.beta != 0.0)
            *dst = (TC)(val + d.beta * (double)*dst);
          else
            *dst = (TC)val;
        }
      }
}

// Sum of split-K partials in split order: C[i][j] = sum_s P[s][i][j].  With
// `mirror` (a symmetric product computed on upper tiles only) an element of a
// skipped tile below the diagonal takes its transposed partner.
template <typename TC>
__global__ void reduce_partials_kernel(const double *__restrict__ P, int splits, int64_t M,
                                       int64_t N, TC *__restrict__ C, int64_t ldc, bool mirror) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx / N, j = idx - i * N;
  const int64_t src = (mirror && i / kBM > j / kBN) ? j * N + i : idx;
  double s = 0.0;
  for (int sp = 0; sp < splits; ++sp) s += P[(int64_t)sp * M * N + src];
  C[i * ldc + j] = (TC)s;
}

// C[i][j] = C[j][i] for the elements of tiles below the diagonal.
__global__ void mirror_tiles_kernel(double *__restrict__ C, int64_t n, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  if (i / kBM > j / kBN) C[i * ldc + j] = C[j * ldc + i];
}

}  // namespace

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Whether gemm_launch takes the large-tile kernel for these operands.
template <typename TA, typename TB>
static bool gemm_big_eligible(const GemmDesc &d, const TA *A, const TB *B) {
  const bool b_ok = d.sbj == 1 && d.sbk % 4 == 0 && aligned16(B);
  const bool a_k = d.sak == 1 && d.sai % 4 == 0;
  const bool a_i = d.sai == 1 && d.sak % 4 == 0;
  return b_ok && (a_k || a_i) && aligned16(A) && d.M >= 64 && d.N >= 64;
}

template <typename TA, typename TB, typename TC, bool F64>
static int gemm_launch(const GemmDesc &d, const TA *A, const TB *B, TC *C, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return BSRHT_OK;
  const bool a_k = d.sak == 1 && d.sai % 4 == 0;
  if (gemm_big_eligible(d, A, B)) {
    dim3 grid((unsigned)((d.M + kBM - 1) / kBM), (unsigned)((d.N + kBN - 1) / kBN),
              (unsigned)d.splits);
    if (a_k)
      gemm_big_kernel<TA, TB, TC, F64, true><<<grid, kBThreads, 0, s>>>(d, A, B, C);
    else
      gemm_big_kernel<TA, TB, TC, F64, false><<<grid, kBThreads, 0, s>>>(d, A, B, C);
    BSRHT_LAUNCH_CHECK();
    return BSRHT_OK;
  }
  dim3 grid((unsigned)((d.M + kTM - 1) / kTM), (unsigned)((d.N + kTN - 1) / kTN),
            (unsigned)d.splits);
  gemm_kernel<TA, TB, TC, F64><<<grid, kGemmThreads, 0, s>>>(d, A, B, C);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int gemm_f32(const GemmDesc &d, const float *A, const float *B, float *C, hipStream_t s) {
  return gemm_launch<float, float, float, false>(d, A, B, C, s);
}
int gemm_f64(const GemmDesc &d, const double *A, const double *B, double *C, hipStream_t s) {
  return gemm_launch<double, double, double, true>(d, A, B, C, s);
}
int gemm_f32f64_f64(const GemmDesc &d, const float *A, const double *B, double *C,
                    hipStream_t s) {
  return gemm_launch<float, double, double, true>(d, A, B, C, s);
}
int gemm_f64f64_f32(const GemmDesc &d, const double *A, const double *B, float *C,
                    hipStream_t s) {
  return gemm_launch<double, double, float, true>(d, A, B, C, s);
}
int gemm_f32f32_f64(const GemmDesc &d, const float *A, const float *B, double *C,
                    hipStream_t s) {
  return gemm_launch<float, float, double, true>(d, A, B, C, s);
}

// G = X^T X (K x K, FP64) for X with rows r < n, X[r][c] = X[r*sr + c*sc],
// split over rows into `splits` FP64 partials summed in order.
template <typename TX>
static int gram_impl(const TX *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
                     int64_t ldg, double *partials, int splits, hipStream_t s) {
  GemmDesc d;
  d.M = K;
  d.N = K;
  d.K = n;
  d.sai = sc;  // A = X^T: A[i][k] = X[k][i]
  d.sak = sr;
  d.sbk = sr;  // B = X
  d.sbj = sc;
  d.alpha = 1.0;
  d.beta = 0.0;
  // G is symmetric: when the large-tile kernel runs, only its tiles on or
  // above the diagonal are computed and the rest is mirrored.
  d.upper_tiles = gemm_big_eligible(d, X, X);
  const int64_t total = K * K;
  if (splits <= 1) {
    d.splits = 1;
    d.ldc = ldg;
    d.split_stride = 0;
    int st = gemm_launch<TX, TX, double, true>(d, X, X, G, s);
    if (st != BSRHT_OK || !d.upper_tiles) return st;
    mirror_tiles_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(G, K, ldg);
    BSRHT_LAUNCH_CHECK();
    return BSRHT_OK;
  }
  d.splits = splits;
  d.ldc = K;
  d.split_stride = K * K;
  int st = gemm_launch<TX, TX, double, true>(d, X, X, partials, s);
  if (st != BSRHT_OK) return st;
  reduce_partials_kernel<double><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(
      partials, splits, K, K, G, ldg, d.upper_tiles);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int gram_f32(const float *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
             int64_t ldg, double *partials, int splits, hipStream_t s) {
  return gram_impl<float>(X, n, K, sr, sc, G, ldg, partials, splits, s);
}
int gram_f64(const double *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
             int64_t ldg, double *partials, int splits, hipStream_t s) {
  return gram_impl<double>(X, n, K, sr, sc, G, ldg, partials, splits, s);
}

int64_t gram_partial_elems(int64_t n, int64_t Kmax) {
  int64_t best = 0;
  for (int64_t K = 1; K <= Kmax; ++K) {
    const int64_t sp = gram_splits(n, K);
    if (sp > 1) best = std::max(best, sp * K * K);
  }
  return best;
}

int gram_splits(int64_t n, int64_t K) {
  // at most two workgroups per CU (the FP64 kernel's occupancy) over the tiles
  // on or above the diagonal, so that all of them run in one round; each split
  // spans at least 1024 rows
  const int64_t nt = (K + kBM - 1) / kBM;
  const int64_t tiles = nt * (nt + 1) / 2;
  int64_t want = 2 * (int64_t)device_cu_count() / tiles;
  const int64_t maxs = (n + 1023) / 1024;
  if (want > maxs) want = maxs;
  if (want < 1) want = 1;
  if (want > 256) want = 256;
  return (int)want;
}

namespace {

// ---------------------------------------------------------------------------
// FP64 Cholesky G = C^T C with C upper triangular, in place, blocked
// right-looking with nb x nb diagonal blocks: factor the diagonal block in
// LDS, solve the block row C12 = C11^{-T} G12, update the trailing block
// G22 -= C12^T C12 on the matrix cores.  A pivot <= tol * max(diag(G)) of the
// original G stops the factorisation: its 1-based index goes to *info and the
// later steps do nothing (the Remark 3.1 break-down).
constexpr int kCholNB = 32;

struct CholState {
  double thresh;
  int32_t stop;
};

__global__ __launch_bounds__(256) void chol_init_kernel(const double *__restrict__ G, int64_t n,
                                                        int64_t ldg, double tol,
                                                        CholState *st, int32_t *info) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, G[i * ldg + i]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->thresh = tol * red[0];
    st->stop = 0;
    *info = 0;
  }
}

// Factor the nb x nb diagonal block at (kb, kb) in LDS.
__global__ __launch_bounds__(1024) void chol_diag_kernel(double *G, int64_t ldg, int64_t kb,
                                                         int nb, CholState *st, int32_t *info) {
  __shared__ double T[kCholNB][kCholNB + 1];
  __shared__ int s_fail;
  if (st->stop) return;
  const int tid = threadIdx.x;
  const int r = tid / kCholNB, c = tid % kCholNB;
  if (r < nb && c < nb) T[r][c] = G[(kb + r) * ldg + kb + c];
  if (tid == 0) s_fail = 0;
  __syncthreads();
  const double thresh = st->thresh;
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      const double p = T[k][k];
      if (!(p > thresh))
        s_fail = (int)(kb + k + 1);
      else
        T[k][k] = sqrt(p);
    }
    __syncthreads();
    if (s_fail) break;
    if (r == k && c > k && c < nb) T[k][c] /= T[k][k];
    __syncthreads();
    if (r > k && r < nb && c >= r && c < nb) T[r][c] -= T[k][r] * T[k][c];
    __syncthreads();
  }
  if (s_fail) {
    if (tid == 0) {
      st->stop = 1;
      *info = s_fail;
    }
    return;
  }
  if (r < nb && c < nb) G[(kb + r) * ldg + kb + c] = (c >= r) ? T[r][c] : 0.0;
}

// Block row: C12[:, j] = C11^{-T} G12[:, j] for the columns j right of the
// diagonal block (forward substitution with the lower-triangular C11^T).
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *G, int64_t n, int64_t ldg,
                                                        int64_t kb, int nb, const CholState *st) {
  __shared__ double C11[kCholNB][kCholNB + 1];
  if (st->stop) return;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += blockDim.x) C11[e / nb][e % nb] = G[(kb + e / nb) * ldg + kb + e % nb];
  __syncthreads();
  const int64_t j = kb + nb + (int64_t)blockIdx.x * blockDim.x + tid;
  if (j >= n) return;
  double x[kCholNB];
#pragma unroll
  for (int i = 0; i < kCholNB; ++i) {
    if (i < nb) {
      double s = G[(kb + i) * ldg + j];
#pragma unroll
      for (int t = 0; t < kCholNB; ++t)
        if (t < i) s -= C11[t][i] * x[t];
      x[i] = s / C11[i][i];
      G[(kb + i) * ldg + j] = x[i];
    }
  }
}

// zero the strict lower triangle after a successful factorisation
__global__ void chol_finish_kernel(double *G, int64_t n, int64_t ldg, const CholState *st) {
  if (st->stop) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  if (j < i) G[i * ldg + j] = 0.0;
}

// Inverse of an upper-triangular n x n matrix C (row-major): column j of
// Ci = C^{-1} solves C x = e_j by back substitution; one wave per column, the
// dot product of each step split across the lanes, x kept in LDS.
constexpr int kTrinvWaves = 4;

__global__ __launch_bounds__(64 * kTrinvWaves) void trinv_upper_kernel(
    const double *__restrict__ C, int64_t n, int64_t ldc, double *__restrict__ Ci, int64_t ldi) {
  extern __shared__ double s_x[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * kTrinvWaves + wv;
  double *x = s_x + (int64_t)wv * n;
  if (j >= n) return;
  for (int64_t i = lane; i < n; i += 64) x[i] = 0.0;
  for (int64_t i = j; i >= 0; --i) {
    double s = 0.0;
    for (int64_t t = i + 1 + lane; t <= j; t += 64) s += C[i * ldc + t] * x[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const double xi = (((i == j) ? 1.0 : 0.0) - s) / C[i * ldc + i];
    if (lane == 0) x[i] = xi;
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): x[i] is in LDS before the next step
    __builtin_amdgcn_wave_barrier();
  }
  for (int64_t i = lane; i < n; i += 64) Ci[i * ldi + j] = x[i];
}

// ---------------------------------------------------------------------------
// One-sided block Jacobi (Hestenes) on the columns of X (nr x nc,
// column-major, columns of length nr at stride ldx): columns are rotated in
// pairs until all are mutually orthogonal, X V = U Sigma.  The singular
// values are the final column norms.  Without accumulation the returned
// vectors are the normalised columns (U); a column with small sigma_j then
// carries an error of order u sigma_1 / sigma_j, which is harmless where the
// caller weights column j by sigma_j (the SVD of an R factor, passed as
// X = R^T: the row-major buffer of R already is R^T in column-major order).
// With accumulation (V != NULL) the rotations are also applied to V = I and
// its columns are returned: V stays orthogonal to working precision, so for
// a symmetric X the pairs (v_j, v_j^T X v_j) are a backward-stable eigen
// decomposition, which callers that scale by 1/sqrt(lambda_j) need.
//
// Blocking: the columns form nc/W blocks of W.  One launch is one round of a
// round-robin over block pairs; a workgroup copies its pair (2W columns) into
// LDS and runs one full cyclic sweep over the 2W(2W-1)/2 column pairs there
// (W disjoint pairs at a time, one wave per pair), recording the
// rotations in a 2W x 2W matrix J; it then writes the columns back and, when
// accumulating, updates V's 2W columns as V J.  A sweep is nc/W - 1 launches;
// sweeps repeat until one performs no rotation.
struct JacobiBlockArgs {
  double *X;
  int nr;
  int64_t ldx;
  double *V;  // NULL, or nc x nc column-major (leading dimension nc)
  int nc, nblocks, round;
  double tol;
  const double *floor2;  // (u ||X||_F)^2: columns at or below it are rounding noise
  unsigned int *rot;     // workgroups that rotated in this sweep
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One 32-bit DPP lane permutation applied to both halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF,
                                                            true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL,
                                                            0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Wave-wide sum, identical in every lane: each level adds a value and its
// partner's with the operands swapped between the two lanes, which IEEE
// addition makes bitwise equal.  The first four levels stay inside a row of
// 16 lanes (DPP: quad permutations, half-row and row mirrors); the last two
// cross rows.
__device__ __forceinline__ double wave_sum_fast(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Pair p of round r among nc players (round-robin, player nc-1 fixed).
__device__ __forceinline__ void rr_pair(int nc, int r, int p, int &a, int &b) {
  const int m = nc - 1;
  if (p == 0) {
    a = r % m;
    b = m;
  } else {
    a = (r + p) % m;
    b = (r + m - p) % m;
  }
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
}

// L[c * ldl + i] = src[gcol(c) * lds + i] for the flattened index
// e = c * rows + i < total; eight loads per thread are in flight at once.
template <int NT, class GCol>
__device__ __forceinline__ void copy_in(double *L, int ldl, const double *__restrict__ src,
                                        int64_t lds, int rows, int total, const GCol &gcol) {
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      if (e < total) {
        const int c = e / rows, i = e - c * rows;
        v[u] = src[gcol(c) * lds + i];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      if (e < total) {
        const int c = e / rows, i = e - c * rows;
        L[c * ldl + i] = v[u];
      }
    }
  }
}

template <int W, int KR>
__global__ __launch_bounds__(64 * W) void jacobi_block_kernel(JacobiBlockArgs ja) {
  constexpr int C = 2 * W;            // columns of a block pair
  constexpr int NRMAX = 64 * KR;      // rows held (KR per lane)
  constexpr int LDL = NRMAX + 2;      // LDS column stride (breaks bank aliasing)
  constexpr int NT = 64 * W;          // one wave per column pair of a round
  __shared__ double L[C * LDL];
  __shared__ double J[C * C];         // column-major: J[c * C + k]
  const int tid = threadIdx.x;
  const int nr = ja.nr;
  int ba, bb;
  rr_pair(ja.nblocks, ja.round, (int)blockIdx.x, ba, bb);
  auto gcol = [&](int c) -> int64_t { return c < W ? (int64_t)ba * W + c : (int64_t)bb * W + (c - W); };
  // Copies run over the flattened (column, row) index in batches of 8 loads
  // per thread, issued before any of them is waited for.
  const int total = C * nr;
  copy_in<NT>(L, LDL, ja.X, ja.ldx, nr, total, gcol);
  if (ja.V)
    for (int e = tid; e < C * C; e += NT) J[e] = (e / C == e % C) ? 1.0 : 0.0;
  __syncthreads();
  const int team = tid >> 6, lt = tid & 63;
  const double floor2 = *ja.floor2;
  bool any = false;
  for (int ir = 0; ir < C - 1; ++ir) {
    int ca, cb;
    rr_pair(C, ir, team, ca, cb);
    double *xa = L + ca * LDL, *xb = L + cb * LDL;
    // the pair's rows of this lane, read once and kept for the rotation
    double u[KR], v[KR];
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      const int i = lt + 64 * q;
      u[q] = i < nr ? xa[i] : 0.0;
      v[q] = i < nr ? xb[i] : 0.0;
    }
    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
    for (int q = 0; q < KR; ++q) {
      al += u[q] * u[q];
      be += v[q] * v[q];
      ga += u[q] * v[q];
    }
    al = wave_sum_fast(al);
    be = wave_sum_fast(be);
    ga = wave_sum_fast(ga);
    // A column whose norm is at the rounding level of the whole matrix has no
    // relative accuracy left, so its orthogonality cannot improve: such pairs
    // count as converged (otherwise a rank-deficient input never converges).
    if (fabs(ga) > ja.tol * sqrt(al * be) && ga != 0.0 && fmin(al, be) > floor2) {
      // rotation zeroing the (a, b) entry of the 2x2 Gram [al ga; ga be]
      const double zeta = (be - al) / (2.0 * ga);
      const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
      for (int q = 0; q < KR; ++q) {
        const int i = lt + 64 * q;
        if (i < nr) {
          xa[i] = c * u[q] - sn * v[q];
          xb[i] = sn * u[q] + c * v[q];
        }
      }
      if (ja.V) {
        double *Ja = J + ca * C, *Jb = J + cb * C;
        for (int i = lt; i < C; i += 64) {
          const double u = Ja[i], v = Jb[i];
          Ja[i] = c * u - sn * v;
          Jb[i] = sn * u + c * v;
        }
      }
      any = true;
    }
    __syncthreads();
  }
  for (int e = tid; e < total; e += NT) {
    const int c = e / nr, i = e - c * nr;
    ja.X[gcol(c) * ja.ldx + i] = L[c * LDL + i];
  }
  const bool rotated = __syncthreads_or(any);
  if (ja.V && rotated) {
    // V's block-pair columns <- (those columns) J, staged through LDS
    // (nc <= NRMAX is guaranteed by the host's choice of W)
    copy_in<NT>(L, LDL, ja.V, ja.nc, ja.nc, C * ja.nc, gcol);
    __syncthreads();
    for (int c = 0; c < C; ++c) {
      const double *Jc = J + c * C;
      double *dst = ja.V + gcol(c) * ja.nc;
      for (int i = tid; i < ja.nc; i += NT) {
        double acc = 0.0;
        for (int k = 0; k < C; ++k) acc += L[k * LDL + i] * Jc[k];
        dst[i] = acc;
      }
    }
  }
  if (rotated && tid == 0) atomicAdd(ja.rot, 1u);
}

// sigma_j = ||x_j||; order by decreasing sigma (ties by index) into S, and
// write in that order as the columns of Us either the normalised columns of X
// (row-major nr x nc, zero where sigma = 0) or, when V is given, the columns
// of V (row-major nc x nc).  One workgroup; nc <= 4096.
__global__ __launch_bounds__(1024) void jacobi_finish_kernel(const double *__restrict__ X,
                                                             int64_t nr, int64_t nc, int64_t ldx,
                                                             const double *__restrict__ V,
                                                             int64_t ldv,
                                                             double *__restrict__ S,
                                                             double *__restrict__ Us,
                                                             int64_t ldu, int32_t *__restrict__ perm) {
  extern __shared__ double s_sig[];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int64_t j = tid; j < nc; j += nt) {
    double s = 0.0;
    for (int64_t i = 0; i < nr; ++i) {
      const double u = X[j * ldx + i];
      s += u * u;
    }
    s_sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int64_t j = tid; j < nc; j += nt) {
    const double sj = s_sig[j];
    int64_t rank = 0;
    for (int64_t t = 0; t < nc; ++t) {
      const double st = s_sig[t];
      rank += (st > sj) || (st == sj && t < j);
    }
    perm[rank] = (int32_t)j;
    S[rank] = sj;
  }
  __syncthreads();
  if (V) {
    for (int64_t e = tid; e < nc * nc; e += nt) {
      const int64_t i = e / nc, rnk = e % nc;
      Us[i * ldu + rnk] = V[(int64_t)perm[rnk] * ldv + i];
    }
    return;
  }
  for (int64_t e = tid; e < nr * nc; e += nt) {
    const int64_t i = e / nc, rnk = e % nc;
    const int64_t col = perm[rnk];
    const double sg = s_sig[col];
    Us[i * ldu + rnk] = sg > 0.0 ? X[col * ldx + i] / sg : 0.0;
  }
}

// out = (u ||X||_F)^2, u = 2^-53, for X (nr x nc, column-major, ldx).  One
// workgroup of 1024 threads; fixed summation order.
__global__ __launch_bounds__(1024) void noise_floor_kernel(const double *__restrict__ X,
                                                            int64_t nr, int64_t nc, int64_t ldx,
                                                            double *__restrict__ out) {
  __shared__ double part[16];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int64_t c = w; c < nc; c += 16) {  // wave w: columns w, w + 16, ...
    const double *col = X + c * ldx;
    for (int64_t i = lane; i < nr; i += 64) acc += col[i] * col[i];
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += part[w];
    const double u = 0x1p-53;
    *out = u * u * t;
  }
}

__global__ void or_bits_kernel(int32_t *p, int32_t bits) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p |= bits;
}

__global__ void zero_u32_kernel(unsigned int *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void fill_f64_kernel(double *p, int64_t count, double value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void eye_kernel(double *M, int64_t n, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  M[i * ld + j] = (i == j) ? 1.0 : 0.0;
}

// dst[j][i] = src[i][j] converted, for src rows x cols.
template <typename TS, typename TD>
__global__ void transpose_kernel(const TS *__restrict__ src, int64_t rows, int64_t cols,
                                 int64_t lds, TD *__restrict__ dst, int64_t ldd) {
  __shared__ TS tile[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + r, j = bj + tx;
    if (i < rows && j < cols) tile[r][tx] = src[i * lds + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = bj + r, i = bi + tx;
    if (i < rows && j < cols) dst[j * ldd + i] = (TD)tile[tx][r];
  }
}

// dst[i][j] = src[i][j] * scale[j] (scale may be NULL: plain copy/convert),
// for j < cols_keep, and 0 for cols_keep <= j < cols_out.
template <typename TS, typename TD>
__global__ void scale_cols_kernel(const TS *__restrict__ src, int64_t rows, int64_t cols_keep,
                                  int64_t cols_out, int64_t lds, const double *__restrict__ scale,
                                  TD *__restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols_out) return;
  const int64_t i = idx / cols_out, j = idx % cols_out;
  double v = 0.0;
  if (j < cols_keep) {
    v = (double)src[i * lds + j];
    if (scale) v *= scale[j];
  }
  dst[i * ldd + j] = (TD)v;
}

}  // namespace

int cholesky_upper(double *G, int64_t n, int64_t ldg, double tol, int32_t *info,
                   void *state, hipStream_t s) {
  if (n <= 0) return BSRHT_OK;
  CholState *st = static_cast<CholState *>(state);
  chol_init_kernel<<<1, 256, 0, s>>>(G, n, ldg, tol, st, info);
  BSRHT_LAUNCH_CHECK();
  for (int64_t kb = 0; kb < n; kb += kCholNB) {
    const int nb = (int)std::min<int64_t>(kCholNB, n - kb);
    chol_diag_kernel<<<1, 1024, 0, s>>>(G, ldg, kb, nb, st, info);
    BSRHT_LAUNCH_CHECK();
    const int64_t rest = n - kb - nb;
    if (rest <= 0) break;
    chol_trsm_kernel<<<(unsigned)((rest + 255) / 256), 256, 0, s>>>(G, n, ldg, kb, nb, st);
    BSRHT_LAUNCH_CHECK();
    GemmDesc d;  // G22 -= C12^T C12 (full trailing block; only its upper part is used)
    d.M = rest;
    d.N = rest;
    d.K = nb;
    d.sai = 1;
    d.sak = ldg;
    d.sbk = ldg;
    d.sbj = 1;
    d.ldc = ldg;
    d.alpha = -1.0;
    d.beta = 1.0;
    const double *C12 = G + kb * ldg + kb + nb;
    double *G22 = G + (kb + nb) * ldg + kb + nb;
    int rc = gemm_launch<double, double, double, true>(d, C12, C12, G22, s);
    if (rc != BSRHT_OK) return rc;
  }
  chol_finish_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, s>>>(G, n, ldg, st);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

size_t cholesky_state_bytes() { return sizeof(CholState); }

int fill_f64(double *p, int64_t count, double value, hipStream_t s) {
  if (count <= 0) return BSRHT_OK;
  fill_f64_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(p, count, value);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int trinv_upper(const double *C, int64_t n, int64_t ldc, double *Ci, int64_t ldi, hipStream_t s) {
  if (n <= 0) return BSRHT_OK;
  if (n * kTrinvWaves * sizeof(double) > 64 * 1024) return BSRHT_EUNSUPPORTED;
  trinv_upper_kernel<<<(unsigned)((n + kTrinvWaves - 1) / kTrinvWaves), 64 * kTrinvWaves,
                       (size_t)n * kTrinvWaves * sizeof(double), s>>>(C, n, ldc, Ci, ldi);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int eye(double *M, int64_t n, int64_t ld, hipStream_t s) {
  eye_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, s>>>(M, n, ld);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

// One launch per round, nblocks - 1 rounds per sweep; after each sweep the
// rotation counter is read back and the sweeps stop at the first one without
// rotations.  *sweeps = max_sweeps + 1 when that never happens.
template <int W, int KR>
static Task jacobi_sweeps_task(DevCtx &ctx, JacobiBlockArgs ja, int max_sweeps, int *sweeps) {
  ja.nblocks = ja.nc / W;
  *sweeps = max_sweeps + 1;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    zero_u32_kernel<<<1, 64, 0, ctx.s>>>(ja.rot, 1);
    if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
    for (int r = 0; r < ja.nblocks - 1; ++r) {
      ja.round = r;
      jacobi_block_kernel<W, KR><<<(unsigned)(ja.nblocks / 2), 64 * W, 0, ctx.s>>>(ja);
      if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
    }
    unsigned int rot = 0;
    BSRHT_CO_TRY(co_await readback(ctx, &rot, ja.rot, sizeof(rot)));
    if (rot == 0) {
      *sweeps = sw + 1;
      break;
    }
  }
  co_return BSRHT_OK;
}

// Block width W and rows per lane KR (64 KR >= rows) for a problem whose
// LDS copy holds `rows` rows.  Measured on MI355X (graded 320..1024-column
// problems): narrower blocks give more workgroups per round and win up to
// 512 rows; beyond that the LDS capacity decides.
static void jacobi_shape(int64_t rows, int *W, int *KR) {
  if (rows <= 512) {
    *W = 8;
    *KR = 8;
  } else if (rows <= 1024) {
    *W = 8;
    *KR = 16;
  } else if (rows <= 2048) {
    *W = 4;
    *KR = 32;
  } else {
    *W = 2;
    *KR = 64;
  }
}

Task jacobi_svd_task(DevCtx &ctx, double *X, int64_t nr, int64_t nc, int64_t ldx, double *V,
                     double *S, double *Us, int64_t ldu, int32_t *perm, unsigned int *flags,
                     int max_sweeps, int32_t *info, int W, int KR) {
  if (nc <= 0) co_return BSRHT_OK;
  const int64_t rows = V ? std::max(nr, nc) : nr;
  if (W == 0) jacobi_shape(rows, &W, &KR);
  if (nc > 4096 || nr > 4096 || (nc % 32) != 0 || rows > 64 * (int64_t)KR)
    co_return BSRHT_EUNSUPPORTED;
  hipStream_t s = ctx.s;
  if (V) {
    eye_kernel<<<(unsigned)((nc * nc + 255) / 256), 256, 0, s>>>(V, nc, nc);
    if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  }
  JacobiBlockArgs ja;
  ja.X = X;
  ja.nr = (int)nr;
  ja.ldx = ldx;
  ja.V = V;
  ja.nc = (int)nc;
  ja.nblocks = 0;
  ja.round = 0;
  ja.tol = 1e-15 * (double)(nr > 16 ? nr : 16);
  ja.rot = flags;
  double *floor2 = reinterpret_cast<double *>(flags + 2);
  ja.floor2 = floor2;
  noise_floor_kernel<<<1, 1024, 0, s>>>(X, nr, nc, ldx, floor2);
  if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  int sweeps = 0, st;
  switch (W * 1000 + KR) {
    case 16008: st = co_await jacobi_sweeps_task<16, 8>(ctx, ja, max_sweeps, &sweeps); break;
    case 8008: st = co_await jacobi_sweeps_task<8, 8>(ctx, ja, max_sweeps, &sweeps); break;
    case 8016: st = co_await jacobi_sweeps_task<8, 16>(ctx, ja, max_sweeps, &sweeps); break;
    case 4008: st = co_await jacobi_sweeps_task<4, 8>(ctx, ja, max_sweeps, &sweeps); break;
    case 4016: st = co_await jacobi_sweeps_task<4, 16>(ctx, ja, max_sweeps, &sweeps); break;
    case 4032: st = co_await jacobi_sweeps_task<4, 32>(ctx, ja, max_sweeps, &sweeps); break;
    case 2064: st = co_await jacobi_sweeps_task<2, 64>(ctx, ja, max_sweeps, &sweeps); break;
    default: co_return BSRHT_EUNSUPPORTED;
  }
  if (st != BSRHT_OK) co_return st;
  if (sweeps > max_sweeps && info) {
    or_bits_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_JACOBI_NOCONV);
    if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  }
  jacobi_finish_kernel<<<1, 1024, (size_t)nc * sizeof(double), s>>>(X, nr, nc, ldx, V, nc, S,
                                                                     Us, ldu, perm);
  if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  co_return BSRHT_OK;
}

int jacobi_svd_shape(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
                     double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
                     int32_t *info, int W, int KR, hipStream_t s) {
  DevCtx ctx;
  ctx.s = s;
  return run_blocking(jacobi_svd_task(ctx, X, nr, nc, ldx, V, S, Us, ldu, perm, flags,
                                      max_sweeps, info, W, KR));
}

int jacobi_svd(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
               double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
               int32_t *info, hipStream_t s) {
  return jacobi_svd_shape(X, nr, nc, ldx, V, S, Us, ldu, perm, flags, max_sweeps, info, 0, 0, s);
}

int transpose_f32_f64(const float *src, int64_t rows, int64_t cols, int64_t lds, double *dst,
                      int64_t ldd, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  transpose_kernel<float, double><<<grid, 256, 0, s>>>(src, rows, cols, lds, dst, ldd);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}
int transpose_f32(const float *src, int64_t rows, int64_t cols, int64_t lds, float *dst,
                  int64_t ldd, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  transpose_kernel<float, float><<<grid, 256, 0, s>>>(src, rows, cols, lds, dst, ldd);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}
int transpose_f64(const double *src, int64_t rows, int64_t cols, int64_t lds, double *dst,
                  int64_t ldd, hipStream_t s) {
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  transpose_kernel<double, double><<<grid, 256, 0, s>>>(src, rows, cols, lds, dst, ldd);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

template <typename TS, typename TD>
static int scale_cols_impl(const TS *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                           const double *scale, TD *dst, int64_t ldd, hipStream_t s) {
  const int64_t total = rows * out;
  if (total <= 0) return BSRHT_OK;
  scale_cols_kernel<TS, TD><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(
      src, rows, keep, out, lds, scale, dst, ldd);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}
int scale_cols_f64_f32(const double *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                       const double *scale, float *dst, int64_t ldd, hipStream_t s) {
  return scale_cols_impl<double, float>(src, rows, keep, out, lds, scale, dst, ldd, s);
}
int scale_cols_f64(const double *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                   const double *scale, double *dst, int64_t ldd, hipStream_t s) {
  return scale_cols_impl<double, double>(src, rows, keep, out, lds, scale, dst, ldd, s);
}
int scale_cols_f32(const float *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                   const double *scale, float *dst, int64_t ldd, hipStream_t s) {
  return scale_cols_impl<float, float>(src, rows, keep, out, lds, scale, dst, ldd, s);
}

}  // namespace bsrht
