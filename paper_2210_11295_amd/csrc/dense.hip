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
#include <climits>

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

// A symmetric product on upper tiles computes the tiles on or above the
// diagonal, and in a diagonal tile not the lower-left quadrant (the wave that
// owns it skips its matrix-core work, which frees its SIMD for the other
// workgroup there); the skipped elements are mirrored from their partners.
__host__ __device__ inline bool upper_tiles_skipped(int64_t i, int64_t j) {
  const int64_t ti = i / kBM, tj = j / kBN;
  return ti > tj || (ti == tj && i % kBM >= kBM / 2 && j % kBN < kBN / 2);
}

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
  // Tile order: workgroups are dealt to the 8 XCDs round-robin by linear id
  // L, so L runs tile (L mod 8) * (G / 8) + L / 8 of the grid's natural order
  // (G a multiple of 8, else unchanged): each XCD takes a contiguous range,
  // whose tiles share their row and column panels (and, for split-K, the
  // rows of their k range) through that XCD's L2.
  const int gx = gridDim.x, gy = gridDim.y;
  const int64_t G = (int64_t)gx * gy * gridDim.z;
  const int64_t L = blockIdx.x + (int64_t)gx * (blockIdx.y + (int64_t)gy * blockIdx.z);
  const int64_t lt = (G & 7) == 0 ? (L & 7) * (G >> 3) + (L >> 3) : L;
  const int bxr = (int)(lt % gx), byr = (int)((lt / gx) % gy), bzr = (int)(lt / ((int64_t)gx * gy));
  if (d.upper_tiles && bxr > byr) return;  // mirrored by the caller
  const int64_t i0 = (int64_t)bxr * kBM, j0 = (int64_t)byr * kBN;
  int64_t kchunk = (d.K + gridDim.z - 1) / gridDim.z;
  kchunk = (kchunk + KT - 1) / KT * KT;
  const int64_t kb = (int64_t)bzr * kchunk;
  const int64_t ke = min(d.K, kb + kchunk);
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  // lower-left quadrant of a diagonal tile of a symmetric product (uniform
  // per wave): the wave still moves its share of the tiles through LDS
  const bool quad_skip = d.upper_tiles && bxr == byr && wi > wj;
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
    for (int ks = 0; ks < (quad_skip ? 0 : KT); ks += 4) {
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
  TC *Cz = C + (int64_t)bzr * d.split_stride;
  if (quad_skip) return;
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M * N;
       idx += stride) {
    const int64_t i = idx / N, j = idx - i * N;
    const int64_t src = (mirror && upper_tiles_skipped(i, j)) ? j * N + i : idx;
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += P[(int64_t)sp * M * N + src];
    C[i * ldc + j] = (TC)s;
  }
}

// C[i][j] = C[j][i] for the elements an upper-tile product skipped.
__global__ void mirror_tiles_kernel(double *__restrict__ C, int64_t n, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx - i * n;
  if (upper_tiles_skipped(i, j)) C[i * ldc + j] = C[j * ldc + i];
}

// ---------------------------------------------------------------------------
// Gram of a tall FP32 matrix on the int8 matrix cores, exact to FP64 level.
// Column c of X is scaled by 2^-e_c (|x| < 2^e_c over the column) and written
// in seven signed base-128 digits by round-to-nearest,
//   x = 2^(e_c - 6) * sum_{a<7} d_a 2^(-7a) + rem,  |d_a| <= 64,
//   |rem| <= 2^(e_c - 49) (half the last digit's unit),
// so x_i x_j = 2^(e_i + e_j - 12) sum_{a,b} d_a d'_b 2^(-7(a+b)).  The digit
// products are exact in int32 (v_mfma_i32_16x16x64_i8); the 28 pairs with
// a + b <= 6 are accumulated per level a + b and the levels combined in FP64
// once per row chunk.  A digit of 64 times 64, seven pairs to a level and
// at most kI8MaxChunk rows keep every level below 2^31.  Elements at least
// 2^-24 of their column's maximum are represented exactly, the dropped pairs
// sit below 2^-49 of the column maxima's product: the error is at the level
// of an FP64 accumulation of the exact products.
constexpr int kI8Digits = 7;
constexpr int kI8T = 64;      // output tile (and column block) width
constexpr int kI8Rows = 64;   // rows per step
constexpr int64_t kI8MaxChunk = 65536;
constexpr int kI8NonFinite = 1 << 20;  // column exponent marking an Inf / NaN column

using I4 = int __attribute__((ext_vector_type(4)));

// part[b][c] = max |X[r][c]| (as float bits, NaN above Inf above finite) over
// the rows of block b.
__global__ __launch_bounds__(256) void colmax_partial_kernel(const float *__restrict__ X,
                                                             int64_t n, int64_t K, int64_t sr,
                                                             int64_t rows_per,
                                                             unsigned *__restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = min(n, r0 + rows_per);
  for (int64_t c = threadIdx.x; c < K; c += blockDim.x) {
    unsigned m = 0;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) m = max(m, __float_as_uint(X[r * sr + c]) & 0x7fffffffu);
    part[(int64_t)blockIdx.x * K + c] = m;
  }
}

// ex[c]: the exponent e with max |X[.][c]| < 2^e (0 for a zero column,
// kI8NonFinite for a column holding Inf or NaN).  64 columns per workgroup,
// the partials' blocks shared by 16 groups of 64 threads.
__global__ __launch_bounds__(1024) void colexp_kernel(const unsigned *__restrict__ part,
                                                      int blocks, int64_t K,
                                                      int *__restrict__ ex) {
  __shared__ unsigned red[16][64];
  const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + cl;
  unsigned m = 0;
  if (c < K) {
#pragma unroll 8
    for (int b = grp; b < blocks; b += 16) m = max(m, part[(int64_t)b * K + c]);
  }
  red[grp][cl] = m;
  __syncthreads();
  if (grp != 0 || c >= K) return;
  for (int r = 1; r < 16; ++r) m = max(m, red[r][cl]);
  int e = 0;
  if (m >= 0x7f800000u)
    e = kI8NonFinite;
  else if (m != 0)
    (void)frexpf(__uint_as_float(m), &e);
  ex[c] = e;
}

struct I8GramArgs {
  const float *X;
  int64_t n, K, sr;
  int64_t rows_per;  // rows per split, a multiple of kI8Rows, <= kI8MaxChunk
  const int *ex;
  double *P;  // [splits][K][K] FP64 partials
  int nt;     // column blocks of kI8T
  int tiles;  // nt (nt + 1) / 2 tiles on or above the diagonal
  int items;  // tiles * splits
};

// Byte offset of the 16-row group g of column col in a digit plane: 64 bytes
// per column, the groups XOR-swizzled by column so that any 8 (and any 16)
// consecutive lanes of a 128-bit read hit distinct banks.
__device__ __forceinline__ int i8_off(int col, int g) {
  return col * kI8Rows + 16 * (g ^ (((col >> 1) ^ (col >> 3)) & 3));
}

// One workgroup: a 64 x 64 tile of partial G over the rows of one split.
// Wave w owns rows 16w..16w+15 of the tile and all four 16-column subtiles.
__global__ __launch_bounds__(256) void gram_i8_kernel(I8GramArgs g) {
  __shared__ __attribute__((aligned(16))) unsigned char sl[2][kI8Digits][kI8T * kI8Rows];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // consecutive workgroups go round-robin over the eight XCDs: give each XCD
  // a contiguous run of work items (split-major), so that the tiles of one
  // row range share that XCD's L2
  int w = (int)blockIdx.x;
  if (g.items % 8 == 0) w = (w % 8) * (g.items / 8) + w / 8;
  const int split = w / g.tiles;
  int t = w - split * g.tiles, bi = 0;
  while (t >= g.nt - bi) {
    t -= g.nt - bi;
    ++bi;
  }
  const int bj = bi + t;
  const bool diag = bi == bj;
  const int64_t ci0 = (int64_t)bi * kI8T, cj0 = (int64_t)bj * kI8T;
  const int64_t rb = (int64_t)split * g.rows_per;
  const int64_t re = min(g.n, rb + g.rows_per);
  const int steps = re > rb ? (int)((re - rb + kI8Rows - 1) / kI8Rows) : 0;

  // loader: column c of the block, rows 16q..16q+15 of a step (one 16-row
  // group of the digit planes, written with one 128-bit store per digit).
  // A column past K reads column K-1 instead: it only reaches outputs past
  // K, which are not stored.  Buffer loads over the split's rows: the
  // descriptor's range check returns 0 for rows past its end.
  const int c = lane, q = wave;
  const int64_t coli = min(ci0 + c, g.K - 1), colj = min(cj0 + c, g.K - 1);
  const int ei = g.ex[coli], ej = g.ex[colj];
  const int shi = ei == kI8NonFinite ? 0 : 6 - ei;
  const int shj = ej == kI8NonFinite ? 0 : 6 - ej;
  const int sr4 = (int)g.sr * 4;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(g.X + rb * g.sr), 0, re > rb ? (int)((re - rb) * sr4) : 0,
      0x00020000);
  const int vi = 16 * q * sr4 + 4 * (int)coli, vj = 16 * q * sr4 + 4 * (int)colj;
  float xi[16], xj[16];
  auto load = [&](int step) {
    const int so = step * kI8Rows * sr4;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int o = so + u * sr4;
      // (on a diagonal tile xj repeats xi's column and is not converted)
      xi[u] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vi + o, 0, 0));
      xj[u] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vj + o, 0, 0));
    }
  };
  // digits of 16 values (rows 16q..16q+15 of column c) into the planes of
  // buffer b
  auto convert = [&](const float *x, int sh, int b) {
    float r[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) r[u] = ldexpf(x[u], sh);
    const int off = i8_off(c, q);
#pragma unroll
    for (int a = 0; a < kI8Digits; ++a) {
      const float M = 12582912.0f * __builtin_ldexpf(1.0f, -7 * a);  // 1.5 * 2^(23 - 7a)
      unsigned w[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        unsigned bits[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float tt = r[4 * h + u] + M;  // r rounded to a multiple of 2^-7a, plus M
          bits[u] = __float_as_uint(tt);
          if (a + 1 < kI8Digits) r[4 * h + u] -= tt - M;
        }
        const unsigned p01 = __builtin_amdgcn_perm(bits[1], bits[0], 0x0c0c0400u);
        const unsigned p23 = __builtin_amdgcn_perm(bits[3], bits[2], 0x0c0c0400u);
        w[h] = __builtin_amdgcn_perm(p23, p01, 0x05040100u);
      }
      *reinterpret_cast<uint4 *>(&sl[b][a][off]) = uint4{w[0], w[1], w[2], w[3]};
    }
  };

  I4 acc[4][kI8Digits];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int d = 0; d < kI8Digits; ++d) acc[s][d] = I4{0, 0, 0, 0};

  const int li = lane & 15, lg = lane >> 4;
  const int jb = diag ? 0 : 1;
  if (steps > 0) load(0);
  for (int step = 0; step < steps; ++step) {
    __syncthreads();  // the previous step's reads of the planes are done
    convert(xi, shi, 0);
    if (!diag) convert(xj, shj, 1);
    __syncthreads();
    if (step + 1 < steps) load(step + 1);
    I4 av[kI8Digits];
#pragma unroll
    for (int a = 0; a < kI8Digits; ++a)
      av[a] = *reinterpret_cast<const I4 *>(&sl[0][a][i8_off(16 * wave + li, lg)]);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int b = 0; b < kI8Digits; ++b) {
        const I4 bv = *reinterpret_cast<const I4 *>(&sl[jb][b][i8_off(16 * s + li, lg)]);
#pragma unroll
        for (int a = 0; a + b < kI8Digits; ++a)
          acc[s][a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[a], bv, acc[s][a + b], 0, 0, 0);
      }
  }

  // D[4 lg + v][li] of subtile s: G[ci0 + 16 wave + 4 lg + v][cj0 + 16 s + li]
  double *P = g.P + (int64_t)split * g.K * g.K;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t i = ci0 + 16 * wave + 4 * lg + v;
    if (i >= g.K) continue;
    const int eri = g.ex[i];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t j = cj0 + 16 * s + li;
      if (j >= g.K) continue;
      const int erj = g.ex[j];
      double val;
      if (eri == kI8NonFinite || erj == kI8NonFinite) {
        val = __builtin_nan("");
      } else {
        val = 0.0;
#pragma unroll
        for (int d = kI8Digits - 1; d >= 0; --d)
          val += ldexp((double)acc[s][d][v], eri + erj - 12 - 7 * d);
      }
      P[i * g.K + j] = val;
    }
  }
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
static int gemm_launch(const GemmDesc &d, const TA *A, const TB *B, TC *C, hipStream_t s,
                       bool small_tiles = false) {
  if (d.M <= 0 || d.N <= 0) return BSRHT_OK;
  const bool a_k = d.sak == 1 && d.sai % 4 == 0;
  if (!small_tiles && gemm_big_eligible(d, A, B)) {
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

int gemm_f32_splitk(const GemmDesc &d0, const float *A, const float *B, float *C,
                    double *partials, int splits, hipStream_t s) {
  if (d0.M <= 0 || d0.N <= 0) return BSRHT_OK;
  if (splits <= 1) return gemm_f32(d0, A, B, C, s);
  GemmDesc d = d0;
  d.splits = splits;
  d.split_stride = d.M * d.N;
  d.ldc = d.N;
  d.alpha = 1.0;
  d.beta = 0.0;
  BSRHT_TRY((gemm_launch<float, float, double, false>(d, A, B, partials, s)));
  const int64_t total = d.M * d.N;
  reduce_partials_kernel<float><<<stride_grid(total, 256), 256, 0, s>>>(
      partials, splits, d.M, d.N, C, d0.ldc, false);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
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
  reduce_partials_kernel<double><<<stride_grid(total, 256), 256, 0, s>>>(
      partials, splits, K, K, G, ldg, d.upper_tiles);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

// Whether gram_f32 takes the int8 path (gram_i8_kernel): a tall X with unit
// column stride; *s8 row splits (at most the caller's `splits`, whose
// partials buffer they use, and enough for kI8MaxChunk rows each) and *cmb
// column-max blocks.
constexpr int64_t kI8MinRows = 16384;
static bool gram_i8_shape(int64_t n, int64_t K, int64_t sr, int64_t sc, int splits, int *s8,
                          int *cmb) {
  if (sc != 1 || sr < K || n < kI8MinRows || K < 1 || K > 4096 || splits < 2) return false;
  const int64_t nt = (K + kI8T - 1) / kI8T, tiles = nt * (nt + 1) / 2;
  const int64_t need = (n + kI8MaxChunk - 1) / kI8MaxChunk;
  // two rounds of two workgroups per CU
  int64_t want = std::max<int64_t>(4 * (int64_t)device_cu_count() / tiles, need);
  want = std::min<int64_t>({want, (int64_t)splits, (n + kI8Rows - 1) / kI8Rows});
  if (want < need || tiles * want > INT_MAX) return false;
  // byte offsets within a split's rows are 32-bit
  const int64_t rows_per = ((n + want - 1) / want + kI8Rows - 1) / kI8Rows * kI8Rows;
  if (rows_per * sr * 4 > INT_MAX) return false;
  *s8 = (int)want;
  *cmb = (int)std::min<int64_t>({1024, 2 * K - 1, n});
  return true;
}

// G = X^T X through int8 digit planes.  The column exponents and the
// column-max partials are kept in G itself (K + cmb*K <= 2 K^2 words) until
// the reduction of the split partials overwrites it.
static int gram_i8(const float *X, int64_t n, int64_t K, int64_t sr, double *G, int64_t ldg,
                   double *partials, int s8, int cmb, hipStream_t s) {
  int *ex = reinterpret_cast<int *>(G);
  unsigned *part = reinterpret_cast<unsigned *>(G) + K;
  const int64_t rows_cm = (n + cmb - 1) / cmb;
  const int blocks = (int)((n + rows_cm - 1) / rows_cm);
  colmax_partial_kernel<<<blocks, 256, 0, s>>>(X, n, K, sr, rows_cm, part);
  BSRHT_LAUNCH_CHECK();
  colexp_kernel<<<(unsigned)((K + 63) / 64), 1024, 0, s>>>(part, blocks, K, ex);
  BSRHT_LAUNCH_CHECK();
  I8GramArgs a;
  a.X = X;
  a.n = n;
  a.K = K;
  a.sr = sr;
  a.rows_per = ((n + s8 - 1) / s8 + kI8Rows - 1) / kI8Rows * kI8Rows;
  a.ex = ex;
  a.P = partials;
  a.nt = (int)((K + kI8T - 1) / kI8T);
  a.tiles = a.nt * (a.nt + 1) / 2;
  a.items = a.tiles * s8;
  gram_i8_kernel<<<a.items, 256, 0, s>>>(a);
  BSRHT_LAUNCH_CHECK();
  // the 64-wide tiles cover every element the 128-wide upper-tile reduction reads
  reduce_partials_kernel<double><<<stride_grid(K * K, 256), 256, 0, s>>>(
      partials, s8, K, K, G, ldg, true);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int gram_f32(const float *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
             int64_t ldg, double *partials, int splits, hipStream_t s) {
  int s8 = 0, cmb = 0;
  if (gram_i8_shape(n, K, sr, sc, splits, &s8, &cmb))
    return gram_i8(X, n, K, sr, G, ldg, partials, s8, cmb, s);
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
// dot product of each step split across the lanes, x kept in LDS.  Lane q
// holds the entries t = i+1+q+64u of row i of C in registers (addresses
// clamped into the row; entries past j meet x[j + 1], which stays zero).
// Rows arrive through a ring of DEPTH register buffers, each refilled right
// after its step with the row DEPTH steps further on: a step waits only on a
// load issued DEPTH steps earlier.  The dot product is summed by DPP into
// lane 63.  A step has no lane-dependent branch (every lane stores x_i, lane
// 63 into x and the others into a pad), so the reciprocal of the next row's
// diagonal, formed during the current step, stays off its dependent chain and
// each step multiplies instead of dividing.
// x moved across lanes by one DPP control (32-bit halves): a lane without a
// source reads 0 (bound_ctrl), a lane outside row_mask gets 0.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROW_MASK, 0xF, BOUND);
  return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over the wave, left in lane 63 (other lanes hold partial sums): pairs
// and quads by quad_perm, rows of 16 by row_shr 4 and 8, then row 0's sum
// broadcast into rows 1 and 3 and row 1's into rows 2 and 3 (row_bcast 15 and
// 31).  Six dependent DPP steps where a 64-bit shuffle reduction takes six
// round trips through the LDS permute unit.
__device__ __forceinline__ double wave_sum_to_lane63(double s) {
  s += dpp_f64<0xb1, 0xF, true>(s);   // quad_perm [1, 0, 3, 2]
  s += dpp_f64<0x4e, 0xF, true>(s);   // quad_perm [2, 3, 0, 1]
  s += dpp_f64<0x114, 0xF, true>(s);  // row_shr 4
  s += dpp_f64<0x118, 0xF, true>(s);  // row_shr 8
  s += dpp_f64<0x142, 0xA, false>(s); // row_bcast 15 into rows 1 and 3
  s += dpp_f64<0x143, 0xC, false>(s); // row_bcast 31 into rows 2 and 3
  return s;
}

// LDS doubles per wave: x (n + 1, x[n] = 0) and the 64-entry pad.
__host__ __device__ inline size_t trinv_lds_doubles(int64_t n) { return (size_t)n + 1 + 64; }

template <int PER, int WAVES>  // n <= 64 * PER; WAVES columns per workgroup
__global__ __launch_bounds__(64 * WAVES) void trinv_upper_kernel(
    const double *__restrict__ C, int64_t n, int64_t ldc, double *__restrict__ Ci, int64_t ldi) {
  constexpr int DEPTH = PER <= 16 ? 4 : 2;
  extern __shared__ double s_x[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * WAVES + wv;
  double *x = s_x + (int64_t)wv * (int64_t)trinv_lds_doubles(n);
  if (j >= n) return;
  for (int64_t i = lane; i <= n; i += 64) x[i] = 0.0;
  double *const xout = lane == 63 ? x : x + n + 1 + lane;  // where this lane stores x_i
  auto load_row = [&](int64_t i, double (&v)[PER], double &d) {
    const double *row = C + i * ldc;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t t = i + 1 + lane + 64 * u;
      v[u] = row[t <= j ? t : j];
    }
    d = row[i];
  };
  __builtin_amdgcn_s_waitcnt(0xc07f);  // the zeros are in LDS before the first step
  __builtin_amdgcn_wave_barrier();
  // slot k holds row j - k, then j - k - DEPTH, ... (rows below 0 read row 0)
  double ring[DEPTH][PER], dg[DEPTH];
#pragma unroll
  for (int k = 0; k < DEPTH; ++k) load_row(j - k >= 0 ? j - k : 0, ring[k], dg[k]);
  double rcur = 1.0 / dg[0];
  for (int64_t i0 = j; i0 >= 0; i0 -= DEPTH) {
#pragma unroll
    for (int k = 0; k < DEPTH; ++k) {
      const int64_t i = i0 - k;  // wave-uniform
      if (i < 0) break;
      const double rnext = 1.0 / dg[(k + 1) % DEPTH];  // row i - 1's diagonal
      double s = 0.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int64_t t = i + 1 + lane + 64 * u;
        s = fma(ring[k][u], x[t <= j ? t : j + 1], s);
      }
      s = wave_sum_to_lane63(s);
      const double xi = (((i == j) ? 1.0 : 0.0) - s) * rcur;
      xout[lane == 63 ? i : 0] = xi;
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): x[i] is in LDS before the next step
      __builtin_amdgcn_wave_barrier();
      load_row(i - DEPTH >= 0 ? i - DEPTH : 0, ring[k], dg[k]);
      rcur = rnext;
    }
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
// round-robin over block pairs; a workgroup forms the Gram matrix of its pair
// (2W columns), runs rounds of W disjoint 2x2 rotations on it, recording the
// rotations in a 2W x 2W matrix J, and then updates the pair's columns of X
// (and, when accumulating, of V) as X J.  The general form runs one cyclic
// sweep over all 2W(2W-1)/2 column pairs at every meeting; the 16-column form
// does so in round 0 of a sweep only, where every block meets a partner, and
// rotates the W^2 cross pairs alone in the other rounds (the intra-block
// pairs would otherwise be met nc/W - 1 times per sweep; a model of both
// orders on the Nystrom and R-factor problems ends in the same number of
// sweeps, give or take one).  Every column pair is thus tested at least once
// per sweep.  A sweep is nc/W - 1 launches; sweeps repeat until one performs
// no rotation, or (16-column form) until one in which every rotated pair was
// within 1e-8 of orthogonal, which leaves nothing the next sweep would rotate.
struct JacobiBlockArgs {
  double *X;
  int nr;
  int64_t ldx;
  double *V;  // NULL, or nc x nc column-major (leading dimension nc)
  int nc, nblocks, round;
  double tol;
  const double *floor2;  // (u ||X||_F)^2: columns at or below it are rounding noise
  // Per-workgroup slots, cleared before each sweep: workgroup b of every
  // launch of the sweep owns slot b and only ever sets it (plain stores
  // replace atomics on one address, which all workgroups of a launch would
  // otherwise contend for).  rot[b]: workgroup b rotated in this sweep;
  // big[b] (16-column form): it rotated a pair with g_ab^2 / (g_aa g_bb) at
  // or above kJacobiStopOff2.
  unsigned int *rot;
  unsigned int *big;
};

// Stop threshold of the 16-column form, (1e-8)^2 (see jacobi_sweeps_task).
constexpr double kJacobiStopOff2 = 1e-16;


__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
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

// Block width of the Gram form (block pairs of 2W columns).
constexpr int kJacobiGramW = 16;

// Gram form of the block step, for any row count.  The workgroup forms the
// 2W x 2W Gram matrix G = X_p^T X_p of its column pair on FP64 matrix cores,
// runs the cyclic sweep of 2x2 rotations on G itself (a rotation's decision
// and angle use the same three entries -- two squared norms and an inner
// product -- that the column form computes from the columns; after it G is
// updated as J^T G J instead of being recomputed), and applies the
// accumulated rotation to the 2W columns of X (and of V) as one matrix
// product.  Every launch starts from a freshly formed G, so a sweep without
// rotations has tested the inner products of the columns themselves.
template <int W>
__global__ __launch_bounds__(256) void jacobi_gram_kernel(JacobiBlockArgs ja) {
  constexpr int C = 2 * W;                // columns of a block pair
  static_assert(C == 16 || C == 32, "block pairs of 16 or 32 columns");
  constexpr int NB = C / 16;              // 16-column blocks of the MFMA tiles
  constexpr int NUP = NB * (NB + 1) / 2;  // Gram tiles on or above the diagonal
  constexpr int NT = 256;
  constexpr int LG = C + 1;               // LDS row stride of G and J
  constexpr int U = 8;                    // 4-row steps per batch of loads
  using D4 = double __attribute__((ext_vector_type(4)));
  __shared__ double Gs[2][C * LG];
  __shared__ double Js[2][C * LG];
  __shared__ double part[4][NUP][256];
  __shared__ double cself[C], cpart[C], dg[C];
  __shared__ int pidx[C], rotc[C];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int nr = ja.nr;
  int ba, bb;
  rr_pair(ja.nblocks, ja.round, (int)blockIdx.x, ba, bb);
  auto gcol = [&](int c) -> int64_t { return c < W ? (int64_t)ba * W + c : (int64_t)bb * W + (c - W); };

  // 1. G = X_p^T X_p.  A 16x16x4 MFMA takes A[i][k] = X_p[r + k][16 bi + i]
  // and B[k][j] = X_p[r + k][16 bj + j]: lane (k = lane / 16, i = j = lane % 16)
  // supplies the same element to both.  Wave w sums a contiguous quarter of
  // the 4-row steps; the quarters are added in wave order.
  {
    const double *xcol[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) xcol[b] = ja.X + gcol(16 * b + lc) * ja.ldx;
    D4 acc[NUP];
#pragma unroll
    for (int u = 0; u < NUP; ++u) acc[u] = D4{0, 0, 0, 0};
    const int nsteps = (nr + 3) >> 2;
    const int per = (nsteps + 3) >> 2;
    const int s_beg = wave * per, s_end = min(nsteps, s_beg + per);
    for (int s0 = s_beg; s0 < s_end; s0 += U) {
      double x[U][NB];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int row = 4 * (s0 + u) + lr;
        const bool in = s0 + u < s_end && row < nr;
#pragma unroll
        for (int b = 0; b < NB; ++b) x[u][b] = in ? xcol[b][row] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        int t = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj, ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u][bi], x[u][bj], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int u = 0; u < NUP; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) part[wave][u][v * 64 + lane] = acc[u][v];
  }
  for (int e = tid; e < C * LG; e += NT) Js[0][e] = (e / LG == e % LG) ? 1.0 : 0.0;
  __syncthreads();
  for (int e = tid; e < NUP * 256; e += NT) {
    const int u = e >> 8, r = e & 255, v = r >> 6, ln = r & 63;
    int bi = 0, bj = 0, t = 0;
    for (int a = 0; a < NB; ++a)
      for (int b = a; b < NB; ++b, ++t)
        if (t == u) { bi = a; bj = b; }
    const int i = 16 * bi + (ln >> 4) + 4 * v, j = 16 * bj + (ln & 15);
    if (bi == bj && i > j) continue;  // the diagonal tiles' upper halves are mirrored
    const double s = ((part[0][u][r] + part[1][u][r]) + part[2][u][r]) + part[3][u][r];
    Gs[0][i * LG + j] = s;
    Gs[0][j * LG + i] = s;
  }
  __syncthreads();

  // 2. One cyclic sweep over the 2W(2W-1)/2 pairs on G, W disjoint pairs per
  // round, accumulating J.
  const double floor2 = *ja.floor2;
  bool any = false;
  int cur = 0;
  for (int ir = 0; ir < C - 1; ++ir) {
    if (tid < C / 2) {
      int a, b;
      rr_pair(C, ir, tid, a, b);
      const double *G = Gs[cur];
      const double al = G[a * LG + a], be = G[b * LG + b], ga = G[a * LG + b];
      double c = 1.0, sn = 0.0, t = 0.0;
      bool rot = false;
      // A column whose norm is at the rounding level of the whole matrix has
      // no relative accuracy left, so its orthogonality cannot improve: such
      // pairs count as converged (otherwise a rank-deficient input never
      // converges).
      if (fabs(ga) > ja.tol * sqrt(al * be) && ga != 0.0 && fmin(al, be) > floor2) {
        // rotation zeroing the (a, b) entry of the 2x2 Gram [al ga; ga be]
        const double zeta = (be - al) / (2.0 * ga);
        t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        c = 1.0 / sqrt(1.0 + t * t);
        sn = c * t;
        rot = true;
      }
      // column a of the rotation is c e_a - sn e_b, column b is sn e_a + c e_b
      pidx[a] = b;
      pidx[b] = a;
      cself[a] = c;
      cpart[a] = -sn;
      cself[b] = c;
      cpart[b] = sn;
      dg[a] = -t * ga;  // the new diagonal: al - t ga and be + t ga
      dg[b] = t * ga;
      rotc[a] = rot;
      rotc[b] = rot;
      any |= rot;
    }
    __syncthreads();
    const double *G = Gs[cur];
    const double *J = Js[cur];
    double *G2 = Gs[cur ^ 1];
    double *J2 = Js[cur ^ 1];
    for (int e = tid; e < C * C; e += NT) {
      const int i = e / C, j = e - (e / C) * C;
      const int pi = pidx[i], pj = pidx[j];
      if (i <= j) {
        double g;
        if (rotc[i] && j == i)
          g = G[i * LG + i] + dg[i];
        else if (rotc[i] && j == pi)
          g = 0.0;
        else
          g = cself[i] * (cself[j] * G[i * LG + j] + cpart[j] * G[i * LG + pj]) +
              cpart[i] * (cself[j] * G[pi * LG + j] + cpart[j] * G[pi * LG + pj]);
        G2[i * LG + j] = g;
        G2[j * LG + i] = g;
      }
      J2[i * LG + j] = cself[j] * J[i * LG + j] + cpart[j] * J[i * LG + pj];
    }
    __syncthreads();
    cur ^= 1;
  }
  const bool rotated = __syncthreads_or(any);
  if (!rotated) return;

  // 3. X_p <- X_p J (and V_p <- V_p J), 16 rows at a time on matrix cores:
  // A[i][k] = P[16 rb + i][4 ks + k] (lane: i = lane % 16, k = lane / 16),
  // B[k][j] = J[4 ks + k][16 cb + j]; the result's lane holds rows
  // 16 rb + lane / 16 + 4 v of column 16 cb + lane % 16.  A wave reads all 2W
  // columns of its rows before it writes them back.
  const double *J = Js[cur];
  double jb[C / 4][NB];
#pragma unroll
  for (int ks = 0; ks < C / 4; ++ks)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) jb[ks][cb] = J[(4 * ks + lr) * LG + 16 * cb + lc];
  auto apply = [&](double *P, int64_t ld, int rows) {
    double *pin[C / 4];
    double *pout[NB];
#pragma unroll
    for (int ks = 0; ks < C / 4; ++ks) pin[ks] = P + gcol(4 * ks + lr) * ld;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) pout[cb] = P + gcol(16 * cb + lc) * ld;
    const int nrb = (rows + 15) >> 4;
    for (int rb0 = wave; rb0 < nrb; rb0 += 8) {
      double a[2][C / 4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = 16 * (rb0 + 4 * h) + lc;
        const bool in = rb0 + 4 * h < nrb && row < rows;
#pragma unroll
        for (int ks = 0; ks < C / 4; ++ks) a[h][ks] = in ? pin[ks][row] : 0.0;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int rb = rb0 + 4 * h;
        if (rb >= nrb) break;
        D4 d[NB];
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          d[cb] = D4{0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < C / 4; ++ks)
            d[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][ks], jb[ks][cb], d[cb], 0, 0, 0);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * rb + lr + 4 * v;
            if (row < rows) pout[cb][row] = d[cb][v];
          }
      }
    }
  };
  apply(ja.X, ja.ldx, nr);
  if (ja.V) apply(ja.V, ja.nc, ja.nc);
  if (tid == 0) ja.rot[blockIdx.x] = 1u;
}

// The Gram form for block pairs of 16 columns with at most 1024 rows (and V
// of at most 1024 rows), where the block step is bound by latencies:
//  - the pair's columns are read from global memory once, all loads in
//    flight, into LDS (column-major, stride 1026 doubles, which keeps both
//    the Gram reads and the update reads to at most two-way bank conflicts;
//    rows past nr are zero), and V's 16 columns are prefetched into
//    registers in the layout of the update;
//  - a round of the sweep has one barrier: while 256 threads apply round r's
//    rotations to G and J, eight threads of another wave form the three
//    entries of G that round r + 1's pairs need (with the same arithmetic as
//    the full update) and compute round r + 1's rotations;
//  - the update is formed transposed on the matrix cores, so the results
//    leave the accumulators as 128-byte runs of consecutive rows.
constexpr int kJg16Rows = 1024, kJg16Ld = 1026;

struct JgRound {  // round r's rotations, per column (16 columns)
  double cself[16], cpart[16], dg[16];
  int rotc[16];
};

// Partner of column x in round r of the round-robin over 16 columns (the
// pairing rr_pair(16, r, .) makes): 15 meets r, any other x meets
// 2r - x mod 15.
__device__ __forceinline__ int jg_partner(int r, int x) {
  if (x == 15) return r;
  if (x == r) return 15;
  const int y = 2 * r - x;
  return y < 0 ? y + 15 : (y >= 15 ? y - 15 : y);
}

// Inner rounds of a pair step.  Full: the cyclic order over all 16 columns
// (15 rounds, rr_pair(16, r, .)).  Cross: the 64 pairs of a column of the
// first block with one of the second (8 rounds; round r pairs column x < 8
// with column 8 + ((x + r) mod 8)).
__device__ __forceinline__ void jg_pair(bool full, int r, int p, int &a, int &b) {
  if (full) {
    rr_pair(16, r, p, a, b);
  } else {
    a = p;
    b = 8 + ((p + r) & 7);
  }
}

__device__ __forceinline__ int jg_part(bool full, int r, int x) {
  if (full) return jg_partner(r, x);
  return x < 8 ? 8 + ((x + r) & 7) : ((x - r) & 7);
}

// Entry (i, j) of J_r^T G J_r from the round's rotation coefficients of
// columns i and j (cs: on the column itself, cp: on its partner) and the four
// entries of G it combines; an entry of a rotated pair's own 2x2 block is set
// by the rotation's closed form instead.
__device__ __forceinline__ double jg_entry(double csi, double cpi, double csj, double cpj,
                                           int roti, double dgi, bool diag, bool pair,
                                           double gij, double gipj, double gpij, double gpipj) {
  // explicit fused operations: every thread that forms an entry rounds it alike
  const double g = fma(csi, fma(csj, gij, cpj * gipj), cpi * fma(csj, gpij, cpj * gpipj));
  return roti ? (diag ? gij + dgi : (pair ? 0.0 : g)) : g;
}

// The convergence test of pair (a, b): |g_ab| > tol sqrt(g_aa g_bb), taken on
// the squares (tol2 = tol^2), which keeps a square root off the critical path
// of the sweep (G's entries are squared column norms and inner products of
// the columns, far from overflow when squared for any matrix of FP32-range
// entries); a column at the rounding level of the whole matrix counts as
// converged.
__device__ __forceinline__ bool jg_needs_rotation(double al, double be, double ga, double tol2,
                                                  double floor2) {
  return ga * ga > tol2 * (al * be) && ga != 0.0 && fmin(al, be) > floor2;
}

// The rotation of pair (a, b) from the entries al = g_aa, be = g_bb, ga = g_ab.
// Its tangent only decides how far the (a, b) entry drops, so it is formed in
// FP32: t = 2 ga sgn(d) / (|d| + sqrt(d^2 + 4 ga^2)), d = be - al (the smaller
// root of t^2 + 2 zeta t - 1 = 0, zeta = d / (2 ga)), with d and 2 ga first
// scaled by the power of two that brings the larger into [1, 2), so neither
// overflows and the smaller underflows only where the pair cannot rotate.
// The entry then drops to ~2e-7 of its size, and the pair's next meeting
// takes the rest.  c = 1/sqrt(1 + t^2) is refined from its FP32 value to FP64
// by two Newton steps and s = c t, so c^2 + s^2 = 1 to working precision and
// the accumulated J stays orthogonal.  This chain is the sweep's critical
// path: FP64 division and square root would take several times longer.
__device__ __forceinline__ void jg_set_rotation(JgRound &P, int a, int b, double al, double be,
                                                double ga, double tol2, double floor2,
                                                bool &any) {
  const bool rot = jg_needs_rotation(al, be, ga, tol2, floor2);
  const double d = be - al, g2 = 2.0 * ga;
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(d), fabs(g2)));
  const float df = (float)ldexp(d, -e), gf = (float)ldexp(g2, -e);
  const float h = __builtin_amdgcn_sqrtf(fmaf(df, df, gf * gf));
  const float tf = (df < 0.f ? -gf : gf) * __builtin_amdgcn_rcpf(fabsf(df) + h);
  const float cf = __builtin_amdgcn_rsqf(fmaf(tf, tf, 1.f));
  const double tr = (double)tf;
  const double hx = 0.5 * fma(tr, tr, 1.0);
  double cr = (double)cf;
  cr = fma(cr, fma(-hx * cr, cr, 0.5), cr);
  cr = fma(cr, fma(-hx * cr, cr, 0.5), cr);
  const double t = rot ? tr : 0.0, c = rot ? cr : 1.0, sn = rot ? cr * tr : 0.0;
  // column a of the rotation is c e_a - sn e_b, column b is sn e_a + c e_b;
  // the new diagonal entries are al - t ga and be + t ga
  P.cself[a] = c;
  P.cpart[a] = -sn;
  P.cself[b] = c;
  P.cpart[b] = sn;
  P.dg[a] = -t * ga;
  P.dg[b] = t * ga;
  P.rotc[a] = rot;
  P.rotc[b] = rot;
  any |= rot;
}

template <bool FULL>
__global__ __launch_bounds__(512) void jacobi_gram16_kernel(JacobiBlockArgs ja) {
  constexpr int W = 8, C = 16, NT = 512, LG = C + 1, NW = NT / 64;
  constexpr int LD = kJg16Ld;
  constexpr int XH = kJg16Rows / NT;          // rows per thread and column (2)
  constexpr int RBW = kJg16Rows / 16 / NW;    // 16-row blocks per wave (8)
  constexpr int PT = 256;                     // first thread of the pair wave
  using D4 = double __attribute__((ext_vector_type(4)));
  __shared__ double Xs[C * LD];
  __shared__ double Gs[2][C * LG];
  __shared__ double Js[2][C * LG];
  __shared__ double part[NW][256];
  __shared__ JgRound Ps[2];
  __shared__ int sbig;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int nr = ja.nr, nv = ja.V ? ja.nc : 0;
  int ba, bb;
  rr_pair(ja.nblocks, ja.round, (int)blockIdx.x, ba, bb);
  auto gcol = [&](int c) -> int64_t { return c < W ? (int64_t)ba * W + c : (int64_t)bb * W + (c - W); };

  // 0. X_p into registers (thread: rows tid and tid + 512 of every column),
  // V_p into registers in the update's operand layout: row block
  // wave + 8 q, lane (lr, lc) -> row 16 rb + lc of column 4 ks + lr.
  double xv[C][XH];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double *col = ja.X + gcol(c) * ja.ldx;
#pragma unroll
    for (int h = 0; h < XH; ++h) {
      const int i = tid + NT * h;
      xv[c][h] = i < nr ? col[i] : 0.0;
    }
  }
  double vv[RBW][C / 4];
  if (nv > 0) {
#pragma unroll
    for (int ks = 0; ks < C / 4; ++ks) {
      const double *col = ja.V + gcol(4 * ks + lr) * ja.nc;
#pragma unroll
      for (int q = 0; q < RBW; ++q) {
        const int row = 16 * (wave + NW * q) + lc;
        vv[q][ks] = row < nv ? col[row] : 0.0;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int h = 0; h < XH; ++h) Xs[c * LD + tid + NT * h] = xv[c][h];
  for (int e = tid; e < C * LG; e += NT) Js[0][e] = (e / LG == e % LG) ? 1.0 : 0.0;
  if (tid == 0) sbig = 0;
  __syncthreads();

  // 1. G = X_p^T X_p on matrix cores (A[i][k] = B[k][j]^T: lane (k, i) holds
  // row 4 s + k of column i); wave w sums the steps s = w mod 8 into two
  // accumulators, the waves' sums are added in wave order.
  {
    constexpr int U = 8;
    D4 acc0 = D4{0, 0, 0, 0}, acc1 = D4{0, 0, 0, 0};
    const int nsteps = (nr + 3) >> 2;
    for (int s0 = wave; s0 < nsteps; s0 += NW * U) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int st = s0 + NW * u;  // rows of steps past nr are zero in Xs
        x[u] = st < nsteps ? Xs[lc * LD + 4 * st + lr] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; u += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], x[u], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u + 1], x[u + 1], acc1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wave][v * 64 + lane] = acc0[v] + acc1[v];
  }
  __syncthreads();
  if (tid < 256) {
    const int v = tid >> 6, ln = tid & 63;
    const int i = (ln >> 4) + 4 * v, j = ln & 15;
    double s = part[0][tid];
#pragma unroll
    for (int w = 1; w < NW; ++w) s += part[w][tid];
    if (i <= j) {
      Gs[0][i * LG + j] = s;
      Gs[0][j * LG + i] = s;
    }
  }
  __syncthreads();

  // A pair step in which every column pair it would rotate (all 120 in a
  // full round, the 64 cross pairs otherwise) passes the convergence test on
  // the freshly formed G makes no rotation (without a rotation G never
  // changes within the step), so it ends here: the last sweep of a run, and
  // the converged pairs of the sweeps before it, cost the loads and the Gram
  // only.  The test is the one the rounds apply.  The same pass notes whether
  // a pair that needs rotating is still at or above the stop threshold.
  const double floor2 = *ja.floor2, tol2 = ja.tol * ja.tol;
  constexpr bool full = FULL;
  constexpr int nrounds = full ? C - 1 : W;
  {
    bool need = false;
    if (tid < (full ? C * (C - 1) / 2 : W * W)) {
      int a, b;
      if (full) {
        int t = tid;  // pair tid -> (a, b), a < b, in row order
        a = 0;
        while (t >= C - 1 - a) {
          t -= C - 1 - a;
          ++a;
        }
        b = a + 1 + t;
      } else {
        a = tid >> 3;
        b = W + (tid & 7);
      }
      const double *G = Gs[0];
      const double al = G[a * LG + a], be = G[b * LG + b], ga = G[a * LG + b];
      need = jg_needs_rotation(al, be, ga, tol2, floor2);
      if (need && ga * ga >= kJacobiStopOff2 * (al * be)) sbig = 1;  // every writer stores 1
    }
    if (!__syncthreads_or(need)) return;
  }

  // 2. The rounds on G, 8 disjoint pairs per round: in round 0 of a sweep
  // one cyclic pass over all 120 pairs (every block has a partner in round 0,
  // so each intra-block pair is met once per sweep), in the other rounds the
  // 64 cross pairs only.  Every LDS read a thread needs in a round is issued
  // at once: the partners follow from the round number.
  bool any = false;
  if (tid >= PT && tid < PT + C / 2) {
    int a, b;
    jg_pair(full, 0, tid - PT, a, b);
    const double *G = Gs[0];
    jg_set_rotation(Ps[0], a, b, G[a * LG + a], G[b * LG + b], G[a * LG + b], tol2, floor2, any);
  }
  __syncthreads();
  int cur = 0;
  for (int ir = 0; ir < nrounds; ++ir) {
    const JgRound &P = Ps[ir & 1];
    const double *G = Gs[cur];
    if (tid < C * C) {
      const double *J = Js[cur];
      double *G2 = Gs[cur ^ 1];
      double *J2 = Js[cur ^ 1];
      const int i = tid >> 4, j = tid & 15;
      const int pi = jg_part(full, ir, i), pj = jg_part(full, ir, j);
      const double csi = P.cself[i], cpi = P.cpart[i], csj = P.cself[j], cpj = P.cpart[j];
      const double g = jg_entry(csi, cpi, csj, cpj, P.rotc[i], P.dg[i], j == i, j == pi,
                                G[i * LG + j], G[i * LG + pj], G[pi * LG + j], G[pi * LG + pj]);
      const double jn = fma(csj, J[i * LG + j], cpj * J[i * LG + pj]);
      if (i <= j) {
        G2[i * LG + j] = g;
        G2[j * LG + i] = g;
      }
      J2[i * LG + j] = jn;
    } else if (tid >= PT && tid < PT + C / 2 && ir + 1 < nrounds) {
      // the next round's pair (a, b) needs entries (a, a), (b, b), (a, b) of
      // the updated G: formed here exactly as the threads above form them
      // (G is stored exactly symmetric, so g_{pa,a} = g_{a,pa}).  All reads
      // are issued before the arithmetic: this chain sets the round's length.
      int a, b;
      jg_pair(full, ir + 1, tid - PT, a, b);
      const int pa = jg_part(full, ir, a), pb = jg_part(full, ir, b);
      const double csa = P.cself[a], cpa = P.cpart[a], csb = P.cself[b], cpb = P.cpart[b];
      const int rota = P.rotc[a], rotb = P.rotc[b];
      const double dga = P.dg[a], dgb = P.dg[b];
      const double gaa = G[a * LG + a], gapa = G[a * LG + pa], gpapa = G[pa * LG + pa];
      const double gbb = G[b * LG + b], gbpb = G[b * LG + pb], gpbpb = G[pb * LG + pb];
      const double gab = G[a * LG + b], gapb = G[a * LG + pb], gpab = G[pa * LG + b],
                   gpapb = G[pa * LG + pb];
      const double al = jg_entry(csa, cpa, csa, cpa, rota, dga, true, false, gaa, gapa, gapa, gpapa);
      const double be = jg_entry(csb, cpb, csb, cpb, rotb, dgb, true, false, gbb, gbpb, gbpb, gpbpb);
      const double ga = jg_entry(csa, cpa, csb, cpb, rota, dga, false, b == pa, gab, gapb, gpab,
                                 gpapb);
      jg_set_rotation(Ps[(ir + 1) & 1], a, b, al, be, ga, tol2, floor2, any);
    }
    __syncthreads();
    cur ^= 1;
  }
  const bool rotated = __syncthreads_or(any);
  if (!rotated) return;

  // 3. X_p <- X_p J and V_p <- V_p J on matrix cores, 16 rows per product,
  // formed transposed, D = J^T P^T: A[i][k] = J[4 ks + k][i] (lane (k, i)),
  // B[k][j] = P[16 rb + j][4 ks + k] (lane (k, j)), so the result's lane
  // (g, j) holds row 16 rb + j of columns g + 4 v.  Each store of a wave then
  // writes 16 consecutive rows of four columns (128-byte runs) straight from
  // the accumulators, with no pass through LDS.
  const double *J = Js[cur];
  double jb[C / 4];
#pragma unroll
  for (int ks = 0; ks < C / 4; ++ks) jb[ks] = J[(4 * ks + lr) * LG + lc];
  auto update_store = [&](const double (&a)[RBW][C / 4], double *P, int64_t ldp, int rows) {
    D4 d[RBW];
#pragma unroll
    for (int q = 0; q < RBW; ++q) d[q] = D4{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < C / 4; ++ks)
#pragma unroll
      for (int q = 0; q < RBW; ++q)
        d[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(jb[ks], a[q][ks], d[q], 0, 0, 0);
#pragma unroll
    for (int q = 0; q < RBW; ++q) {
      const int row = 16 * (wave + NW * q) + lc;
      if (row < rows)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[gcol(lr + 4 * v) * ldp + row] = d[q][v];
    }
  };
  {
    double xa[RBW][C / 4];  // rows past nr are zero in Xs
#pragma unroll
    for (int q = 0; q < RBW; ++q)
#pragma unroll
      for (int ks = 0; ks < C / 4; ++ks)
        xa[q][ks] = Xs[(4 * ks + lr) * LD + 16 * (wave + NW * q) + lc];
    update_store(xa, ja.X, ja.ldx, nr);
  }
  if (nv > 0) update_store(vv, ja.V, ja.nc, nv);
  if (tid == 0) {
    ja.rot[blockIdx.x] = 1u;
    if (sbig) ja.big[blockIdx.x] = 1u;
  }
}

// The end of a Jacobi run, in three launches over the whole chip:
//  1. N[j] = sigma_j = ||x_j|| (one wave per column, fixed summation order);
//  2. S in decreasing order of sigma (ties by index; a NaN norm ranks last),
//     perm[rank] = j; every workgroup stages all of N (nc <= 4096) in LDS;
//  3. the columns of Us in that order: the normalised columns of X (row-major
//     nr x nc, zero where sigma = 0) or, when V is given, the columns of V
//     (row-major nc x nc).
constexpr int kFinishMaxN = 4096;
__global__ __launch_bounds__(256) void col_norms_kernel(const double *__restrict__ X, int64_t nr,
                                                        int64_t nc, int64_t ldx,
                                                        double *__restrict__ N) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= nc) return;  // whole waves
  const double *col = X + j * ldx;
  double acc = 0.0;
  for (int64_t i = lane; i < nr; i += 64) acc += col[i] * col[i];
  acc = wave_sum(acc);
  if (lane == 0) N[j] = sqrt(acc);
}

__global__ __launch_bounds__(256) void sigma_order_kernel(const double *__restrict__ N, int64_t nc,
                                                          double *__restrict__ S,
                                                          int32_t *__restrict__ perm) {
  __shared__ double key[kFinishMaxN];
  for (int64_t t = threadIdx.x; t < nc; t += blockDim.x) {
    const double v = N[t];
    key[t] = v == v ? v : -INFINITY;
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  const double kj = key[j];
  int64_t rank = 0;
  for (int64_t t = 0; t < nc; ++t) rank += (key[t] > kj || (key[t] == kj && t < j)) ? 1 : 0;
  perm[rank] = (int32_t)j;
  S[rank] = N[j];
}

__global__ void finish_columns_kernel(const double *__restrict__ X, int64_t nr, int64_t nc,
                                      int64_t ldx, const double *__restrict__ V, int64_t ldv,
                                      const double *__restrict__ S,
                                      const int32_t *__restrict__ perm, double *__restrict__ Us,
                                      int64_t ldu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (V) {
    if (e >= nc * nc) return;
    const int64_t i = e / nc, rnk = e - i * nc;
    Us[i * ldu + rnk] = V[(int64_t)perm[rnk] * ldv + i];
    return;
  }
  if (e >= nr * nc) return;
  const int64_t i = e / nc, rnk = e - i * nc;
  const double sg = S[rnk];
  Us[i * ldu + rnk] = sg > 0.0 ? X[(int64_t)perm[rnk] * ldx + i] / sg : 0.0;
}

// out = (u ||X||_F)^2, u = 2^-53, for X (nr x nc, column-major, ldx), in two
// launches with a fixed summation order: kFloorBlocks partial sums (block b,
// wave w: columns 4 b + w, 4 b + w + 4 kFloorBlocks, ...) into P, then their
// sum in index order.
constexpr int kFloorBlocks = 32;
__global__ __launch_bounds__(256) void noise_floor_partial_kernel(const double *__restrict__ X,
                                                                  int64_t nr, int64_t nc,
                                                                  int64_t ldx,
                                                                  double *__restrict__ P) {
  __shared__ double part[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * 4 + w; c < nc; c += 4 * kFloorBlocks) {
    const double *col = X + c * ldx;
    for (int64_t i = lane; i < nr; i += 64) acc += col[i] * col[i];
  }
  acc = wave_sum(acc);
  if (lane == 0) part[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) P[blockIdx.x] = ((part[0] + part[1]) + part[2]) + part[3];
}

__global__ void noise_floor_finish_kernel(const double *__restrict__ P, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int b = 0; b < kFloorBlocks; ++b) t += P[b];
  const double u = 0x1p-53;
  *out = u * u * t;
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < rows * cols_out;
       idx += stride) {
    const int64_t i = idx / cols_out, j = idx % cols_out;
    double v = 0.0;
    if (j < cols_keep) {
      v = (double)src[i * lds + j];
      if (scale) v *= scale[j];
    }
    dst[i * ldd + j] = (TD)v;
  }
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
    // a rank-nb update of at most a few thousand rows: the 64 x 64 tiles
    // give four times the workgroups of the large tiles
    int rc = gemm_launch<double, double, double, true>(d, C12, C12, G22, s, true);
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
  if (n > 64 * 32) return BSRHT_EUNSUPPORTED;
  // four columns per workgroup up to n = 1024, two beyond (LDS <= 34 KiB)
  const int waves = n <= 64 * 16 ? 4 : 2;
  const size_t lds = trinv_lds_doubles(n) * waves * sizeof(double);
  const unsigned grid = (unsigned)((n + waves - 1) / waves);
  if (n <= 64 * 8)
    trinv_upper_kernel<8, 4><<<grid, 64 * 4, lds, s>>>(C, n, ldc, Ci, ldi);
  else if (n <= 64 * 16)
    trinv_upper_kernel<16, 4><<<grid, 64 * 4, lds, s>>>(C, n, ldc, Ci, ldi);
  else
    trinv_upper_kernel<32, 2><<<grid, 64 * 2, lds, s>>>(C, n, ldc, Ci, ldi);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

int eye(double *M, int64_t n, int64_t ld, hipStream_t s) {
  eye_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, s>>>(M, n, ld);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

// One launch per round, nblocks - 1 rounds per sweep; after each sweep the
// workgroups' slots are read back and the sweeps stop at the first one
// without rotations.  The 16-column form (LDS16) also stops after a sweep in
// which every rotated pair had g_ab^2 / (g_aa g_bb) below kJacobiStopOff2 =
// 1e-16 before its rotation: such a sweep leaves each pair at most about nc * 1e-16 from
// orthogonal (each later rotation of a column moves the pair's inner product
// by at most the product of two such cosines), below the test tol of
// 1e-15 * max(nr, 16) that a further sweep would apply, so that sweep, which
// would rotate nothing, is not run.  *sweeps = max_sweeps + 1 when neither
// happens.  LDS16 selects the LDS-staged kernel for 16-column block pairs
// (W = 8).
template <int W, bool LDS16>
static Task jacobi_sweeps_task(DevCtx &ctx, JacobiBlockArgs ja, int max_sweeps, int *sweeps) {
  ja.nblocks = ja.nc / W;
  *sweeps = max_sweeps + 1;
  if (ja.nblocks / 2 > kJacobiMaxGroups) co_return BSRHT_EUNSUPPORTED;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // slots 0 .. groups-1 of rot and of big (contiguous, see jacobi_svd_task)
    const int groups = ja.nblocks / 2;
    zero_u32_kernel<<<(unsigned)((2 * kJacobiMaxGroups + 255) / 256), 256, 0, ctx.s>>>(
        ja.rot, 2 * kJacobiMaxGroups);
    if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
    for (int r = 0; r < ja.nblocks - 1; ++r) {
      ja.round = r;
      if constexpr (LDS16) {
        if (r == 0)
          jacobi_gram16_kernel<true><<<(unsigned)groups, 512, 0, ctx.s>>>(ja);
        else
          jacobi_gram16_kernel<false><<<(unsigned)groups, 512, 0, ctx.s>>>(ja);
      } else {
        jacobi_gram_kernel<W><<<(unsigned)groups, 256, 0, ctx.s>>>(ja);
      }
      if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
    }
    // both slot arrays in one copy (they are contiguous)
    unsigned int slots[2 * kJacobiMaxGroups];
    BSRHT_CO_TRY(co_await readback(ctx, slots, ja.rot, sizeof(slots)));
    bool any = false, big = false;
    for (int b = 0; b < groups; ++b) {
      any |= slots[b] != 0;
      big |= slots[kJacobiMaxGroups + b] != 0;
    }
    if (!any || (LDS16 && !big)) {
      *sweeps = sw + 1;
      break;
    }
  }
  co_return BSRHT_OK;
}

Task jacobi_svd_task(DevCtx &ctx, double *X, int64_t nr, int64_t nc, int64_t ldx, double *V,
                     double *S, double *Us, int64_t ldu, int32_t *perm, unsigned int *flags,
                     int max_sweeps, int32_t *info, int form) {
  if (nc <= 0) co_return BSRHT_OK;
  const int64_t rows = V ? std::max(nr, nc) : nr;
  if (form == 0) form = rows <= kJg16Rows ? 1 : 2;
  if (nc > 4096 || nr > 4096 || (nc % 32) != 0 || form < 1 || form > 2 ||
      (form == 1 && rows > kJg16Rows))
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
  // flags: [0..1] floor2, then G rotation slots and G threshold slots
  // (G = kJacobiMaxGroups)
  double *floor2 = reinterpret_cast<double *>(flags);
  ja.rot = flags + 2;
  ja.big = flags + 2 + kJacobiMaxGroups;
  ja.floor2 = floor2;
  // S is written only at the end of the run: it holds the noise floor's
  // partial sums (nc >= 32 = kFloorBlocks) until then
  noise_floor_partial_kernel<<<kFloorBlocks, 256, 0, s>>>(X, nr, nc, ldx, S);
  noise_floor_finish_kernel<<<1, 64, 0, s>>>(S, floor2);
  if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  int sweeps = 0, st;
  if (form == 1)
    st = co_await jacobi_sweeps_task<8, true>(ctx, ja, max_sweeps, &sweeps);
  else
    st = co_await jacobi_sweeps_task<kJacobiGramW, false>(ctx, ja, max_sweeps, &sweeps);
  if (st != BSRHT_OK) co_return st;
  if (sweeps > max_sweeps && info) {
    or_bits_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_JACOBI_NOCONV);
    if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  }
  // Us is written only by the last launch: its first nc entries hold the
  // unsorted norms until then
  col_norms_kernel<<<(unsigned)((nc + 3) / 4), 256, 0, s>>>(X, nr, nc, ldx, Us);
  sigma_order_kernel<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(Us, nc, S, perm);
  const int64_t nout = V ? nc * nc : nr * nc;
  finish_columns_kernel<<<(unsigned)((nout + 255) / 256), 256, 0, s>>>(X, nr, nc, ldx, V, nc, S,
                                                                       perm, Us, ldu);
  if (hipGetLastError() != hipSuccess) co_return BSRHT_EDEVICE;
  co_return BSRHT_OK;
}

int jacobi_svd_shape(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
                     double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
                     int32_t *info, int form, hipStream_t s) {
  DevCtx ctx;
  ctx.s = s;
  return run_blocking(jacobi_svd_task(ctx, X, nr, nc, ldx, V, S, Us, ldu, perm, flags,
                                      max_sweeps, info, form));
}

int jacobi_svd(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
               double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
               int32_t *info, hipStream_t s) {
  return jacobi_svd_shape(X, nr, nc, ldx, V, S, Us, ldu, perm, flags, max_sweeps, info, 0, s);
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
  scale_cols_kernel<TS, TD><<<stride_grid(total, 256), 256, 0, s>>>(
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
