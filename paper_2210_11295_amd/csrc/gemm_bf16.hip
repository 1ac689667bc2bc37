// Tall FP32 products C = A B on the BF16 matrix cores with split operands,
// for the two passes of the randomized SVD (section 3.1, Algorithm 1) that
// stream a tall factor: Z = A Q and U = Z M.
//
// Every FP32 value x is split into BF16 parts, x = x0 + x1 (+ x2), each part
// the round-to-nearest BF16 of what the earlier parts leave (the differences
// are exact in FP32).  A product of two BF16 values is exact in FP32, and
// v_mfma_f32_16x16x32_bf16 accumulates in FP32, so
//   two parts:   A B ~ A0 B0 + A0 B1 + A1 B0             (~2^-16 relative)
//   three parts: A B ~ A0 B0 + A0 B1 + A1 B0 + A0 B2 + A1 B1 + A2 B0
// where the dropped products are below 2^-24 relative: the three-part form
// matches an FP32 product's accuracy.  On gfx950 one 16x16x32 BF16 MFMA takes
// ~18.5 cycles per SIMD against ~37 for the FP32 16x16x4 form, which does an
// eighth of the work: six BF16 products per 32-long k step still cost 2.7x
// fewer matrix-core cycles than FP32.
//
// Layout: A (M x K) is FP32, row-major with k contiguous; B is split once
// per call into planes Bt[p][j][k] (N rounded up to 128 rows, K to 32, zero
// padded), so that both operands are read along k.  A workgroup computes a
// 128 x 128 tile of C with 4 waves of 64 x 64 (4 x 4 blocks of 16 x 16);
// each 32-long k tile of A is loaded as FP32, split, and staged in LDS as
// planes As[p][row][k] next to Bs[p][col][k], with the next tile's loads in
// flight during the MFMAs.  MFMA operands (probed on the device): A[i][k] in
// lane 16 (k / 8) + i, element k % 8; B[k][j] in lane 16 (k / 8) + j, element
// k % 8; D[i][j] in lane 16 (i / 4) + j, register i % 4.
#include "common.h"
#include "dense.h"

namespace bsrht {
namespace {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kXM = 128, kXN = 128, kXK = 32;
constexpr int kXLd = kXK + 8;  // LDS row stride in BF16 (80 bytes: 16 rows on distinct banks)
constexpr int kXThreads = 256;

// Parts of two values, packed two BF16 per dword (first value low).
template <int NP>
__device__ __forceinline__ void split2(float a, float b, uint32_t (&out)[NP]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const bf16x2_t h = __builtin_convertvector((float2_t){a, b}, bf16x2_t);
    out[p] = __builtin_bit_cast(uint32_t, h);
    a -= __uint_as_float(out[p] << 16);
    b -= __uint_as_float(out[p] & 0xffff0000u);
  }
}

struct XArgs {
  const float *A;
  int64_t lda;
  const __bf16 *Bt;  // planes [NP][Np][Kp]
  int64_t Np, Kp;
  float *C;
  int64_t ldc;
  int64_t M, N, K;
  int64_t ntj;  // column tiles (Np / 128)
};

template <int NP>
__global__ __launch_bounds__(kXThreads, 2) void gemm_bf16x_kernel(XArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[NP][kXM][kXLd];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NP][kXN][kXLd];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  // Tile order: the workgroups are dealt to the 8 XCDs round-robin, so
  // linear id L runs logical tile (L mod 8) * (G / 8) + L / 8 (G = grid size,
  // a multiple of 8): each XCD takes a contiguous range of logical tiles, in
  // which the column tiles of one row tile are adjacent and so share that
  // row tile of A through the XCD's L2.
  const int64_t G = (int64_t)gridDim.x, L = blockIdx.x;
  const int64_t lt = (L & 7) * (G >> 3) + (L >> 3);
  const int64_t i0 = (lt / g.ntj) * kXM, j0 = (lt % g.ntj) * kXN;
  if (i0 >= g.M) return;  // padding tiles of the rounded grid
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  // staging: thread t moves row (t / 2), k half (t % 2) * 16 of both tiles.
  // The loads are branch-free (a branch around them makes the wait-count pass
  // drain every load in flight where the paths join): rows past M read row
  // M - 1 and k past K re-reads the last in-range quad, and such values are
  // zeroed by bit masks.  lda is a multiple of 4 and at least K, so every
  // quad read lies inside its row.
  const int srow = tid >> 1, skh = (tid & 1) * 16;
  const int64_t arow = i0 + srow;
  const bool arow_in = arow < g.M;
  const float *asrc = g.A + (arow_in ? arow : g.M - 1) * g.lda;
  const int64_t klast = ((g.K - 1) >> 2) << 2;  // start of the last quad holding data
  const __bf16 *bsrc = g.Bt + (j0 + srow) * g.Kp + skh;  // Bt rows are padded to Np
  struct RegsA {
    u32x4_t a[4];  // FP32 bits
  };
  struct RegsB {
    u32x4_t b[NP][2];
  };
  auto fetch_a = [&](RegsA &r, int64_t k0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t k = k0 + skh + 4 * v;
      const u32x4_t x = *reinterpret_cast<const u32x4_t *>(asrc + (k < klast ? k : klast));
      // masks, not selects: a select lets the compiler load a lane's value
      // under a branch, and the branch waits for every load in flight
      const int64_t kv = arow_in ? g.K : 0;
      const u32x4_t mk = {k < kv ? ~0u : 0u, k + 1 < kv ? ~0u : 0u, k + 2 < kv ? ~0u : 0u,
                          k + 3 < kv ? ~0u : 0u};
      r.a[v] = x & mk;
    }
  };
  auto fetch_b = [&](RegsB &r, int64_t k0) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        r.b[p][h] = *reinterpret_cast<const u32x4_t *>(bsrc + p * g.Np * g.Kp + k0 + 8 * h);
  };
  auto stage = [&](const RegsA &ra, const RegsB &rb) {
    uint32_t w[4][2][NP];  // [quad][pair][part]
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      split2<NP>(__uint_as_float(ra.a[v][0]), __uint_as_float(ra.a[v][1]), w[v][0]);
      split2<NP>(__uint_as_float(ra.a[v][2]), __uint_as_float(ra.a[v][3]), w[v][1]);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        *reinterpret_cast<u32x4_t *>(&As[p][srow][skh + 8 * h]) =
            (u32x4_t){w[2 * h][0][p], w[2 * h][1][p], w[2 * h + 1][0][p], w[2 * h + 1][1][p]};
        *reinterpret_cast<u32x4_t *>(&Bs[p][srow][skh + 8 * h]) = rb.b[p][h];
      }
    }
  };

  floatx4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_t{0.f, 0.f, 0.f, 0.f};

  const int ko = 8 * (lane >> 4), li = lane & 15;
  // A's parts for the wave's four row blocks stay in registers; B's are read
  // one column block at a time (registers are tight with two fetch sets).
  auto compute = [&]() {
    bf16x8_t av[4][NP];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        av[a][p] = *reinterpret_cast<const bf16x8_t *>(&As[p][wi + 16 * a + li][ko]);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bf16x8_t bv[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        bv[p] = *reinterpret_cast<const bf16x8_t *>(&Bs[p][wj + 16 * b + li][ko]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        floatx4_t c = acc[a][b];
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][1], bv[0], c, 0, 0, 0);
        if constexpr (NP == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][0], bv[2], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][1], bv[1], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a][2], bv[0], c, 0, 0, 0);
        }
        acc[a][b] = c;
      }
    }
  };

  // The next tile's loads are in flight during this tile's MFMAs; the tile
  // index is clamped to the last tile, so the loads are unconditional.
  const int64_t ntiles = (g.K + kXK - 1) / kXK;
  const int64_t tl = ntiles - 1;
  RegsA ra;
  RegsB rb;
  fetch_b(rb, 0);
  fetch_a(ra, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    stage(ra, rb);
    __syncthreads();
    const int64_t tn = (t + 1 < tl ? t + 1 : tl) * kXK;
    fetch_b(rb, tn);
    fetch_a(ra, tn);
    compute();
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t gj = j0 + wj + 16 * b + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + wi + 16 * a + 4 * (lane >> 4) + v;
        if (gi < g.M && gj < g.N) g.C[gi * g.ldc + gj] = acc[a][b][v];
      }
    }
}

// Planes Bt[p][j][k] of B[k][j] (K x N, row stride ldb), zero past K and N.
template <int NP>
__global__ void split_planes_kernel(const float *__restrict__ B, int64_t K, int64_t N,
                                    int64_t ldb, __bf16 *__restrict__ Bt, int64_t Np,
                                    int64_t Kp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Np * Kp) return;
  const int64_t j = idx / Kp, k = idx - j * Kp;
  float x = (j < N && k < K) ? B[k * ldb + j] : 0.f;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const __bf16 h = (__bf16)x;
    Bt[p * Np * Kp + idx] = h;
    x -= (float)h;
  }
}

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

}  // namespace

size_t gemm_bf16x_ws_bytes(int64_t N, int64_t K, int parts) {
  if (parts != 2 && parts != 3) return 0;
  return align256((size_t)parts * (size_t)round_up(N, kXN) * (size_t)round_up(K, kXK) * 2);
}

bool gemm_bf16x_eligible(const float *A, int64_t lda) {
  return lda % 4 == 0 && ((uintptr_t)A & 15) == 0;
}

int gemm_f32_bf16x(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                   int64_t ldc, int64_t M, int64_t N, int64_t K, int parts, void *ws,
                   size_t ws_bytes, hipStream_t s) {
  if (M <= 0 || N <= 0) return BSRHT_OK;
  if ((parts != 2 && parts != 3) || K <= 0 || !gemm_bf16x_eligible(A, lda) ||
      ws_bytes < gemm_bf16x_ws_bytes(N, K, parts) || !ws)
    return BSRHT_EINVAL;
  const int64_t Np = round_up(N, kXN), Kp = round_up(K, kXK);
  __bf16 *Bt = static_cast<__bf16 *>(ws);
  const int64_t total = Np * Kp;
  const unsigned sgrid = (unsigned)((total + 255) / 256);
  if (parts == 3)
    split_planes_kernel<3><<<sgrid, 256, 0, s>>>(B, K, N, ldb, Bt, Np, Kp);
  else
    split_planes_kernel<2><<<sgrid, 256, 0, s>>>(B, K, N, ldb, Bt, Np, Kp);
  BSRHT_LAUNCH_CHECK();
  XArgs g;
  g.A = A;
  g.lda = lda;
  g.Bt = Bt;
  g.Np = Np;
  g.Kp = Kp;
  g.C = C;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.ntj = Np / kXN;
  const int64_t tiles = (M + kXM - 1) / kXM * g.ntj;
  dim3 grid((unsigned)((tiles + 7) / 8 * 8));
  if (parts == 3)
    gemm_bf16x_kernel<3><<<grid, kXThreads, 0, s>>>(g);
  else
    gemm_bf16x_kernel<2><<<grid, kXThreads, 0, s>>>(g);
  BSRHT_LAUNCH_CHECK();
  return BSRHT_OK;
}

}  // namespace bsrht
