// Randomized SVD (section 3.1, Algorithm 1) and Nystrom approximation
// (section 3.2, Algorithm 2) on top of the block SRHT sketch.
//
// Where the paper asks for a QR factorisation (TSQR on a distributed
// machine), one GPU uses Cholesky-QR in FP64: the Gram matrix X^T X of the
// tall factor on the matrix cores, then a Cholesky factor R with
// R^T R = X^T X; orthonormal bases are X R^{-1} (twice, "Cholesky-QR2", for
// the range basis Q).  The small SVDs are one-sided Jacobi in FP64.
//
// Both entry points synchronise their stream to read back a Cholesky flag:
// Remark 3.1's fallback (a square root from an eigendecomposition, keeping
// eigenvalues above tau * lambda_max) changes the sizes of the later steps,
// so the path is chosen on the host.
#include <limits.h>

#include <algorithm>
#include <optional>
#include <vector>

#include "common.h"
#include "dense.h"
#include "task.h"

namespace bsrht {
namespace {

constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24, unit roundoff of FP32 data
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53, FP64 unit roundoff
constexpr int kMaxSweeps = 40;

__global__ void eye_f32_kernel(float *M, int64_t n, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  M[i * ld + j] = (i == j) ? 1.f : 0.f;
}

// Bs = (B + B^T) / 2 in FP64 (Omega Y is symmetric in exact arithmetic).
__global__ void sym_f64_kernel(const float *__restrict__ B, int64_t n, int64_t ldb,
                               double *__restrict__ Bs, int64_t lds) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int64_t i = idx / n, j = idx % n;
  Bs[i * lds + j] = 0.5 * ((double)B[i * ldb + j] + (double)B[j * ldb + i]);
}

// inv[j] = 1/sigma_j for j < keep with sigma_j > rel * sigma_0, else 0; the
// outputs S (FP64, count k) get sigma_j^pw for kept j, else 0.  When a
// requested j < k has no kept value the info word gets RANK_CLAMPED.
__global__ void finish_sigma_kernel(const double *__restrict__ sigma, int64_t avail, int64_t k,
                                    double rel, int pw, double *__restrict__ inv,
                                    double *__restrict__ S, int32_t *__restrict__ info) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double s0 = sigma[0];
  const bool keep = j < avail && sigma[j] > rel * s0 && sigma[j] > 0.0;
  inv[j] = keep ? 1.0 / sigma[j] : 0.0;
  S[j] = keep ? (pw == 2 ? sigma[j] * sigma[j] : sigma[j]) : 0.0;
  if (!keep) atomicOr(info, BSRHT_INFO_RANK_CLAMPED);
}

// lam[j] = sum_i V[i][j] W[i][j] for the columns of V (row-major n x n); with
// W = B V this is v_j^T B v_j, the signed eigenvalues behind the Jacobi
// singular values of a symmetric B.  One wave per column, fixed order.
__global__ __launch_bounds__(256) void col_dots_kernel(const double *__restrict__ V, int64_t ldv,
                                                       const double *__restrict__ W, int64_t ldw,
                                                       int64_t n, double *__restrict__ lam) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;  // whole waves
  double acc = 0.0;
  for (int64_t i = lane; i < n; i += 64) acc += V[i * ldv + j] * W[i * ldw + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) lam[j] = acc;
}

// M[i][i] += c for i < n.
__global__ void add_diag_kernel(double *M, int64_t n, int64_t ld, double c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) M[i * ld + i] += c;
}

// M[i][i] += f * v[0] for a value v[0] computed on the device.
__global__ void add_diag_dev_kernel(double *M, int64_t n, int64_t ld, const double *__restrict__ v,
                                    double f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) M[i * ld + i] += f * v[0];
}

// out[c] = 1 / sqrt(max(ev[e], 1e-300)), e = idx[c] (or c without idx), c < keep:
// the scales Lam_+^{-1/2} of an eigen split.
__global__ void inv_sqrt_kernel(const double *__restrict__ ev, const int32_t *__restrict__ idx,
                                int64_t keep, double *__restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < keep) out[c] = 1.0 / sqrt(fmax(ev[idx ? idx[c] : c], 1e-300));
}

// S[i] = sqrt(S[i]) for S[i] > 0, else 0: singular values from Gram eigenvalues.
__global__ void sqrt_clamp_kernel(double *S, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) S[i] = S[i] > 0.0 ? sqrt(S[i]) : 0.0;
}

// M[i][c] = V[i][idx[c]] * sc[c] for c < keep, 0 for keep <= c < ldm (i < rows).
__global__ void gather_scale_cols_kernel(const double *__restrict__ V, int64_t rows, int64_t ldv,
                                         const int32_t *__restrict__ idx,
                                         const double *__restrict__ sc, int64_t keep,
                                         double *__restrict__ M, int64_t ldm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ldm) return;
  const int64_t i = e / ldm, c = e - i * ldm;
  M[e] = c < keep ? V[i * ldv + idx[c]] * sc[c] : 0.0;
}

// perm[r] = i where r is the rank of G's diagonal entry i in descending order
// (ties by index; a NaN ranks last), i < n: a permutation of 0..n-1.  Every
// workgroup stages the whole diagonal (n <= kMaxOrderN) in LDS.
constexpr int kMaxOrderN = 4096;
__global__ __launch_bounds__(256) void desc_diag_order_kernel(const double *__restrict__ G,
                                                              int64_t n, int64_t ldg,
                                                              int32_t *__restrict__ perm) {
  __shared__ double d[kMaxOrderN];
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = G[j * ldg + j];
    d[j] = v == v ? v : -INFINITY;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double di = d[i];
  int64_t r = 0;
  for (int64_t j = 0; j < n; ++j) r += (d[j] > di || (d[j] == di && j < i)) ? 1 : 0;
  perm[r] = (int32_t)i;
}

// P[r][c] = G[perm[r]][perm[c]] (n x n, leading dimensions ldg and ldp).
__global__ void permute_sym_kernel(const double *__restrict__ G, int64_t n, int64_t ldg,
                                   const int32_t *__restrict__ perm, double *__restrict__ P,
                                   int64_t ldp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e - r * n;
  P[r * ldp + c] = G[(int64_t)perm[r] * ldg + perm[c]];
}

// M[perm[i]][c] = V[i][c] * sc[c] for c < keep, 0 for keep <= c < cols
// (i < rows): the rows of V taken back from the order perm to the original.
__global__ void scale_cols_unpermute_kernel(const double *__restrict__ V, int64_t rows,
                                            int64_t ldv, const int32_t *__restrict__ perm,
                                            const double *__restrict__ sc, int64_t keep,
                                            int64_t cols, double *__restrict__ M, int64_t ldm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, c = e - i * cols;
  M[(int64_t)perm[i] * ldm + c] = c < keep ? V[i * ldv + c] * sc[c] : 0.0;
}

__global__ void or_info_kernel(int32_t *info, int32_t bits) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *info |= bits;
}

__global__ void zero_i32_kernel(int32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Shifted Nystrom.  Sum of squares of the n x l FP32 matrix Y (leading
// dimension ldy) in FP64: kSsqBlocks fixed grid-stride partial sums, then
// one block sums them in order and stores nu = c * sqrt(sum) (c =
// sqrt(n) u_s) at nu[0], so the shift never leaves the device.
constexpr int kSsqBlocks = 1024;
template <typename T>
__global__ void ssq_partial_kernel(const T *__restrict__ Y, int64_t n, int64_t l, int64_t ldy,
                                   double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t total = n * l;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)kSsqBlocks * 256) {
    const int64_t g = e / l, j = e - g * l;
    const double v = (double)Y[g * ldy + j];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void shift_of_kernel(const double *__restrict__ part, double c, double *__restrict__ nu) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < kSsqBlocks; ++b) s += part[b];
  nu[0] = c * sqrt(s);
}

// Y[g][j] += nu * Omega[j][g] (eq. (2.3) entry by entry from the plan's
// tables; block i = g / r, position x = g - i r, D bit at i*rp + x), i.e.
// Y + nu Omega^T = (A + nu I) Omega^T.
__global__ void add_shift_kernel(float *__restrict__ Y, int64_t n, int64_t l, int64_t ldy,
                                 const int32_t *__restrict__ R,
                                 const uint32_t *__restrict__ Dbits,
                                 const uint32_t *__restrict__ Dtbits, int64_t dt_words, int64_t r,
                                 int64_t rp, const double *__restrict__ nu, float inv_sqrt_l) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * l) return;
  const int64_t g = e / l, j = e - g * l;
  const int64_t i = g / r, x = g - i * r;
  const int64_t gd = i * rp + x;
  const uint32_t d = (Dbits[gd >> 5] >> (gd & 31)) & 1u;
  const uint32_t h = (uint32_t)__popc((uint32_t)R[j] & (uint32_t)x) & 1u;
  const uint32_t dt = (Dtbits[i * dt_words + (j >> 5)] >> (j & 31)) & 1u;
  const float om = (d ^ h ^ dt) ? -inv_sqrt_l : inv_sqrt_l;
  Y[g * ldy + j] += (float)nu[0] * om;
}

// lambda_j = max(lambda_j - nu, 0): the eigenvalues of A from those of A + nu I.
__global__ void unshift_kernel(double *__restrict__ lam, int64_t k, const double *__restrict__ nu) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) lam[j] = fmax(lam[j] - nu[0], 0.0);
}

// Size of the small SVD problems: a multiple of 32 (the block Jacobi pairs
// column blocks of up to 16); the padding is zero rows and columns.
inline int64_t svd_pad(int64_t x) { return (x + 31) & ~int64_t(31); }

// Workspace of the small SVD stage for an nc x nc problem (nc even).
template <class A>
struct SvdBufs {
  double *X, *V, *S, *Vs, *inv;
  int32_t *perm;
  unsigned int *flags;
  void take(A &a, int64_t nc, int64_t k) {
    X = a.template take<double>((size_t)(nc * nc));
    V = a.template take<double>((size_t)(nc * nc));
    S = a.template take<double>((size_t)nc);
    Vs = a.template take<double>((size_t)(nc * nc));
    inv = a.template take<double>((size_t)std::max<int64_t>(k, nc));
    perm = a.template take<int32_t>((size_t)nc);
    flags = a.template take<unsigned int>(kJacobiFlagWords);
  }
};

// Allocator that only counts (Sizer) or also hands out pointers (Carve).
struct SizeOnly {
  Sizer sz;
  template <class T>
  T *take(size_t n) {
    sz.take<T>(n);
    return nullptr;
  }
};

// Leading dimensions rounded up to 4 elements: the large-tile GEMM takes
// operands whose rows start at 16-byte boundaries, so every tall product of
// the randomized SVD runs on it whatever l, m and k are (the logical sizes
// are unchanged; padding columns are never read).
inline int64_t ld4(int64_t x) { return (x + 3) & ~int64_t(3); }

// ----------------------------------------------------------------------------
// Randomized SVD workspace layout.

// BF16 parts per operand of the tall products Z = A Q and U = Z M: three
// (FP32-level accuracy) for FP32 plans, two for split-BF16 plans.
inline int tall_product_parts(const bsrht_plan_s *pl) {
  return pl->precision == BSRHT_SPLIT_BF16 ? 2 : 3;
}

// C = A B for the tall products: split-BF16 matrix cores when A's rows are
// 16-byte aligned, else the FP32 matrix-core GEMM.
inline int tall_product(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, int parts, void *ws,
                        size_t ws_bytes, hipStream_t s) {
  if (gemm_bf16x_eligible(A, lda))
    return gemm_f32_bf16x(A, lda, B, ldb, C, ldc, M, N, K, parts, ws, ws_bytes, s);
  GemmDesc d;
  d.M = M; d.N = N; d.K = K;
  d.sai = lda; d.sak = 1;
  d.sbk = ldb; d.sbj = 1;
  d.ldc = ldc;
  return gemm_f32(d, A, B, C, s);
}

template <class A>
struct RsvdWs {
  float *W, *Wt;
  void *apply_ws;
  size_t apply_bytes;
  double *G, *Ginv, *Q1, *G2, *C2inv;
  float *Q32, *Z, *M, *Vk;
  double *gram_part, *Gz;
  int32_t *flag;
  void *chol_state;
  void *xws;  // split BF16 planes of Q, then of M (split-BF16 tall products)
  size_t xws_bytes;
  SvdBufs<A> qb, sv;
  void layout(A &a, const bsrht_plan_s *pl, int64_t m, int64_t k) {
    const int64_t l = pl->l, n = pl->n, lq = std::min(l, m);
    const int64_t l4 = ld4(l), lq4 = ld4(lq), k4 = ld4(k);
    const int parts = tall_product_parts(pl);
    W = a.template take<float>((size_t)(l * m));
    Wt = a.template take<float>((size_t)(m * l4));
    apply_bytes = apply_ws_bytes(pl, m);
    apply_ws = a.template take<char>(apply_bytes);
    G = a.template take<double>((size_t)(l * l));
    Ginv = a.template take<double>((size_t)(l * l4));
    Q1 = a.template take<double>((size_t)(m * l4));
    G2 = a.template take<double>((size_t)(l * l));
    C2inv = a.template take<double>((size_t)(l * l4));
    Q32 = a.template take<float>((size_t)(m * lq4));
    Z = a.template take<float>((size_t)(n * lq4));
    gram_part = a.template take<double>((size_t)std::max(
        {gram_partial_elems(m, l), gram_partial_elems(n, lq), (int64_t)1}));
    Gz = a.template take<double>((size_t)(lq * lq));
    M = a.template take<float>((size_t)(lq * k4));
    Vk = a.template take<float>((size_t)(lq * k4));
    flag = a.template take<int32_t>(4);
    chol_state = a.template take<char>(cholesky_state_bytes());
    xws_bytes = std::max(gemm_bf16x_ws_bytes(lq, m, parts), gemm_bf16x_ws_bytes(k, lq, parts));
    xws = a.template take<char>(xws_bytes);
    qb.take(a, svd_pad(l), l);
    sv.take(a, svd_pad(lq), k);
  }
};

// ----------------------------------------------------------------------------
// Nystrom workspace layout.
template <class A>
struct NysWs {
  float *W, *Y, *B;
  void *apply_ws;
  size_t apply_bytes;
  double *Bs, *Cinv, *Mf, *lam, *Z, *gram_part, *Gz, *Mk;
  int32_t *flag;
  void *chol_state;
  double *ssq;  // kSsqBlocks partial sums, then nu (shifted) or ||B||_F (fallback)
  int32_t *kidx;  // fallback: indices of the kept eigenvalues
  int32_t *zperm;  // Z's columns in descending order of norm
  SvdBufs<A> fb, sv;
  void layout(A &a, const bsrht_plan_s *pl, int64_t k) {
    const int64_t l = pl->l, n = pl->n;
    const int64_t l4 = (l + 3) & ~int64_t(3);  // Z's leading dimension bound
    W = a.template take<float>((size_t)(l * n));
    Y = a.template take<float>((size_t)(n * l));
    B = a.template take<float>((size_t)(l * l));
    apply_bytes = std::max(apply_ws_bytes(pl, n), apply_ws_bytes(pl, l));
    apply_ws = a.template take<char>(apply_bytes);
    Bs = a.template take<double>((size_t)(l * l));
    Cinv = a.template take<double>((size_t)(l * l));
    Mf = a.template take<double>((size_t)(l * l4));
    lam = a.template take<double>((size_t)l);
    Z = a.template take<double>((size_t)(n * l4));
    gram_part = a.template take<double>((size_t)std::max(gram_partial_elems(n, l), (int64_t)1));
    Gz = a.template take<double>((size_t)(l * l));
    Mk = a.template take<double>((size_t)(l * std::max<int64_t>(k, 1)));
    flag = a.template take<int32_t>(4);
    chol_state = a.template take<char>(cholesky_state_bytes());
    ssq = a.template take<double>((size_t)kSsqBlocks + 1);
    kidx = a.template take<int32_t>((size_t)l);
    zperm = a.template take<int32_t>((size_t)l);
    fb.take(a, svd_pad(l), l);
    sv.take(a, svd_pad(l), k);
  }
};

// Right singular vectors of the nc0 x nc0 matrix M given row-major at R
// (ldr).  Factor mode (eigen = false, M an R factor): the row-major buffer of
// M is M^T in column-major order, so the one-sided Jacobi on its columns
// yields the left singular vectors of M^T, i.e. the right singular vectors of
// M, as normalised columns.  Eigen mode (eigen = true, M symmetric): the
// rotations are accumulated and returned, so that the eigenvectors stay
// orthogonal to working precision even for tiny |lambda|, where the callers
// scale by 1/sqrt(lambda).  The problem is zero padded to a multiple of 32;
// the extra zero columns sort last.  Sorted singular values in b.S, vectors
// as columns of b.Vs (row-major, leading dimension nc).
template <class A>
Task small_svd_task(DevCtx &ctx, SvdBufs<A> &b, const double *R, int64_t nc0, int64_t ldr,
                    bool eigen, int32_t *info) {
  const int64_t nc = svd_pad(nc0);
  BSRHT_CO_TRY(fill_f64(b.X, nc * nc, 0.0, ctx.s));
  BSRHT_CO_TRY(scale_cols_f64(R, nc0, nc0, nc0, ldr, nullptr, b.X, nc, ctx.s));  // ld ldr -> nc
  co_return co_await jacobi_svd_task(ctx, b.X, nc, nc, nc, eigen ? b.V : nullptr, b.S, b.Vs, nc,
                                     b.perm, b.flags, kMaxSweeps, info, 0);
}


}  // namespace
}  // namespace bsrht

namespace bsrht {

Task rsvd_task(DevCtx &ctx, const bsrht_plan_s *plan, const float *A, int64_t m, int64_t lda,
               int64_t k, float *U, double *S, float *V, int32_t *info, void *ws,
               size_t ws_bytes) {
  hipStream_t s = ctx.s;
  const int64_t n = plan->n, l = plan->l;
  int64_t lq = std::min(l, m);
  const int64_t l4 = ld4(l), lq4 = ld4(lq), k4 = ld4(k);  // padded leading dimensions
  if (svd_pad(std::max(l, lq)) > 4096) co_return BSRHT_EUNSUPPORTED;
  Carve cv(ws, ws_bytes);
  RsvdWs<Carve> w;
  w.layout(cv, plan, m, k);
  if (cv.overflow) co_return BSRHT_ENOMEM;
  int st;
  zero_i32_kernel<<<1, 64, 0, s>>>(info, 1);
  BSRHT_CO_LAUNCH_CHECK();

  // 1. W = Omega A  (l x m): the paper's Y = A_p Omega^T for A_p = A^T.
  if (plan->precision == BSRHT_SPLIT_BF16)
    st = apply_split_bf16(plan, A, m, lda, w.W, m, w.apply_ws, w.apply_bytes, s);
  else
    st = apply_fp32(plan, A, m, lda, w.W, m, w.apply_ws, w.apply_bytes, s);
  if (st != BSRHT_OK) { debug_report(__FILE__, __LINE__, "step", st); co_return st; }

  // 2. Q = orth(W^T) (m x lq).  l >= m: range(W^T) is all of R^m, Q = I.
  if (l >= m) {
    lq = m;
    eye_f32_kernel<<<(unsigned)((m * m + 255) / 256), 256, 0, s>>>(w.Q32, m, lq4);
    BSRHT_CO_LAUNCH_CHECK();
  } else {
    // Cholesky-QR2 of W^T: G = W W^T, G = C^T C, Q1 = W^T C^{-1}; then again.
    // W^T is formed once (m x l, leading dimension l4) so that the Gram and
    // the product take the large-tile GEMM.
    BSRHT_CO_TRY(transpose_f32(w.W, l, m, m, w.Wt, l4, s));
    const int gs = gram_splits(m, l);
    st = gram_f32(w.Wt, m, l, l4, 1, w.G, l, w.gram_part, gs, s);
    if (st != BSRHT_OK) { debug_report(__FILE__, __LINE__, "step", st); co_return st; }
    BSRHT_CO_TRY(cholesky_upper(w.G, l, l, (double)l * kU64, w.flag, w.chol_state, s));
    int32_t hf = 0;
    BSRHT_CO_TRY(co_await readback(ctx, &hf, w.flag, sizeof(hf)));
    int64_t lk = l;  // columns of Q1
    if (hf == 0) {
      BSRHT_CO_TRY(trinv_upper(w.G, l, l, w.Ginv, l4, s));
      GemmDesc d;
      d.M = m; d.N = l; d.K = l;
      d.sai = l4; d.sak = 1;      // A = W^T
      d.sbk = l4; d.sbj = 1;      // B = C^{-1}
      d.ldc = l4;
      BSRHT_CO_TRY(gemm_f32f64_f64(d, w.Wt, w.Ginv, w.Q1, s));
    } else {
      // W^T is rank deficient (e.g. rank(A) < l): an eigen split of
      // G = W W^T keeps the eigenvalues above l u lambda_max and
      // Q1 = W^T V_+ Lam_+^{-1/2}.
      st = gram_f32(w.Wt, m, l, l4, 1, w.G, l, w.gram_part, gs, s);
      if (st != BSRHT_OK) { debug_report(__FILE__, __LINE__, "step", st); co_return st; }
      BSRHT_CO_TRY(co_await small_svd_task(ctx, w.qb, w.G, l, l, true, info));
      std::vector<double> ev((size_t)l);
      if (co_await readback(ctx, ev.data(), w.qb.S, sizeof(double) * (size_t)l) != BSRHT_OK)
        co_return BSRHT_EDEVICE;
      int64_t keep = 0;
      for (int64_t i = 0; i < l; ++i)
        if (ev[(size_t)i] > (double)l * kU64 * ev[0] && ev[(size_t)i] > 0.0) ++keep;
      if (keep < 1) keep = 1;
      inv_sqrt_kernel<<<(unsigned)((keep + 255) / 256), 256, 0, s>>>(w.qb.S, nullptr, keep,
                                                                    w.qb.inv);
      BSRHT_CO_LAUNCH_CHECK();
      const int64_t nce = svd_pad(l);
      BSRHT_CO_TRY(scale_cols_f64(w.qb.Vs, l, keep, keep, nce, w.qb.inv, w.Ginv, l4, s));
      GemmDesc d;
      d.M = m; d.N = keep; d.K = l;
      d.sai = l4; d.sak = 1;
      d.sbk = l4; d.sbj = 1;
      d.ldc = l4;
      BSRHT_CO_TRY(gemm_f32f64_f64(d, w.Wt, w.Ginv, w.Q1, s));
      lk = keep;
      or_info_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_QB_FALLBACK);
      BSRHT_CO_LAUNCH_CHECK();
    }
    // second pass: G2 = Q1^T Q1, C2, Q = Q1 C2^{-1}
    const int gs2 = gram_splits(m, lk);
    BSRHT_CO_TRY(gram_f64(w.Q1, m, lk, l4, 1, w.G2, lk, w.gram_part, gs2, s));
    BSRHT_CO_TRY(cholesky_upper(w.G2, lk, lk, 1e-14, w.flag + 1, w.chol_state, s));
    int32_t hf2 = 0;
    BSRHT_CO_TRY(co_await readback(ctx, &hf2, w.flag + 1, sizeof(hf2)));
    if (hf2 != 0) {  // Q1 has orthonormal columns to O(eps*kappa^2): should not happen
      debug_report(__FILE__, __LINE__, "second Cholesky-QR pass", BSRHT_EDEVICE);
      co_return BSRHT_EDEVICE;
    }
    BSRHT_CO_TRY(trinv_upper(w.G2, lk, lk, w.C2inv, l4, s));
    GemmDesc d;
    d.M = m; d.N = lk; d.K = lk;
    d.sai = l4; d.sak = 1;
    d.sbk = l4; d.sbj = 1;
    d.ldc = lq4;  // lk <= lq
    BSRHT_CO_TRY(gemm_f64f64_f32(d, w.Q1, w.C2inv, w.Q32, s));
    lq = lk;
  }

  // 3. Z = A Q  (n x lq): the paper's Z = Q^T A_p, transposed; matrix cores.
  const int parts = tall_product_parts(plan);
  {
    const int tslot = timing_begin(BSRHT_TIMING_GEMM_AQ, s);
    st = tall_product(A, lda, w.Q32, lq4, w.Z, lq4, n, lq, m, parts, w.xws, w.xws_bytes, s);
    timing_end(tslot, s);
    if (st != BSRHT_OK) { debug_report(__FILE__, __LINE__, "step", st); co_return st; }
  }
  // 4. R-factor of Z: Gz = Z^T Z (FP64), Gz = R^T R.
  const int gsz = gram_splits(n, lq);
  BSRHT_CO_TRY(gram_f32(w.Z, n, lq, lq4, 1, w.Gz, lq, w.gram_part, gsz, s));
  BSRHT_CO_TRY(cholesky_upper(w.Gz, lq, lq, (double)lq * kU32 * kU32, w.flag + 2, w.chol_state, s));
  int32_t hz = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hz, w.flag + 2, sizeof(hz)));
  int pw;
  if (hz == 0) {
    // 5. SVD of R: R = Ut St Vt^T
    BSRHT_CO_TRY(co_await small_svd_task(ctx, w.sv, w.Gz, lq, lq, false, info));
    pw = 1;
  } else {
    // rank(Z) < lq: Z^T Z = Vt St^2 Vt^T from its eigen decomposition
    BSRHT_CO_TRY(gram_f32(w.Z, n, lq, lq4, 1, w.Gz, lq, w.gram_part, gsz, s));
    BSRHT_CO_TRY(co_await small_svd_task(ctx, w.sv, w.Gz, lq, lq, true, info));
    // the Jacobi values are St^2: take square roots through the scale step
    pw = 0;
  }
  const int64_t nce = svd_pad(lq);
  // singular values of Z (sqrt of the Gram eigenvalues on the fallback path)
  if (pw == 0) {
    sqrt_clamp_kernel<<<(unsigned)((lq + 255) / 256), 256, 0, s>>>(w.sv.S, lq);
    BSRHT_CO_LAUNCH_CHECK();
  }
  // 6. U = Z Vt_k St_k^{-1}, S = St_k, V = Q Vt_k
  finish_sigma_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(
      w.sv.S, lq, k, sqrt((double)lq * kU64), 1, w.sv.inv, S, info);
  BSRHT_CO_LAUNCH_CHECK();
  const int64_t keep = std::min(k, lq);
  BSRHT_CO_TRY(scale_cols_f64_f32(w.sv.Vs, lq, keep, k, nce, w.sv.inv, w.M, k4, s));
  BSRHT_CO_TRY(tall_product(w.Z, lq4, w.M, k4, U, k, n, k, lq, parts, w.xws, w.xws_bytes, s));
  BSRHT_CO_TRY(scale_cols_f64_f32(w.sv.Vs, lq, keep, k, nce, nullptr, w.Vk, k4, s));
  {
    GemmDesc d;
    d.M = m; d.N = k; d.K = lq;
    d.sai = lq4; d.sak = 1;
    d.sbk = k4; d.sbj = 1;
    d.ldc = k;
    BSRHT_CO_TRY(gemm_f32(d, w.Q32, w.Vk, V, s));
  }
  co_return BSRHT_OK;
}

}  // namespace bsrht

using namespace bsrht;

extern "C" {

size_t rsvd_workspace(bsrht_plan_t plan, int64_t m, int64_t k) {
  if (!plan || m < 1 || k < 1) return 0;
  SizeOnly so;
  RsvdWs<SizeOnly> w;
  w.layout(so, plan, m, k);
  return align256(so.sz.used);
}

int rsvd(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, int64_t k, float *U,
         double *S, float *V, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !A || !U || !S || !V || !info || m < 1 || k < 1 || lda < m) return BSRHT_EINVAL;
  if (ws_bytes < rsvd_workspace(plan, m, k) || !ws) return BSRHT_ENOMEM;
  DevCtx ctx;
  ctx.s = (hipStream_t)stream;
  return run_blocking(rsvd_task(ctx, plan, A, m, lda, k, U, S, V, info, ws, ws_bytes));
}

size_t nystrom_workspace(bsrht_plan_t plan, int64_t k) {
  if (!plan || k < 1) return 0;
  SizeOnly so;
  NysWs<SizeOnly> w;
  w.layout(so, plan, k);
  return align256(so.sz.used);
}

}  // extern "C"

namespace bsrht {

// Algorithm 2; with `shifted`, on A + nu I (the sketch Y + nu Omega^T) with nu
// subtracted from the eigenvalues at the end.
// The argument checks are the callers' (nystrom, nystrom_shifted and the
// server's job admission).
Task nystrom_task(DevCtx &ctx, const bsrht_plan_s *plan, const float *A, int64_t lda, int64_t k,
                  float *U, double *lambda, int32_t *info, void *ws, size_t ws_bytes,
                  bool shifted) {
  hipStream_t s = ctx.s;
  const int64_t n = plan->n, l = plan->l;
  if (svd_pad(l) > 4096) co_return BSRHT_EUNSUPPORTED;
  Carve cv(ws, ws_bytes);
  NysWs<Carve> w;
  w.layout(cv, plan, k);
  if (cv.overflow) co_return BSRHT_ENOMEM;
  zero_i32_kernel<<<1, 64, 0, s>>>(info, 1);
  BSRHT_CO_LAUNCH_CHECK();
  auto sketch = [&](const float *X, int64_t mm, int64_t ldx, float *Yo) {
    if (plan->precision == BSRHT_SPLIT_BF16)
      return apply_split_bf16(plan, X, mm, ldx, Yo, mm, w.apply_ws, w.apply_bytes, s);
    return apply_fp32(plan, X, mm, ldx, Yo, mm, w.apply_ws, w.apply_bytes, s);
  };
  // 1. Y = A Omega^T = (Omega A)^T (A symmetric)
  BSRHT_CO_TRY(sketch(A, n, lda, w.W));
  BSRHT_CO_TRY(transpose_f32(w.W, l, n, n, w.Y, l, s));
  if (shifted) {
    if (n * l > kMaxGridItems) co_return BSRHT_EUNSUPPORTED;
    // nu = sqrt(n) u_s ||Y||_F (u_s: unit roundoff of the sketch), Y += nu Omega^T
    const double us = plan->precision == BSRHT_SPLIT_BF16 ? 0x1p-17 : kU32;
    ssq_partial_kernel<float><<<kSsqBlocks, 256, 0, s>>>(w.Y, n, l, l, w.ssq);
    shift_of_kernel<<<1, 64, 0, s>>>(w.ssq, sqrt((double)n) * us, w.ssq + kSsqBlocks);
    add_shift_kernel<<<(unsigned)((n * l + 255) / 256), 256, 0, s>>>(
        w.Y, n, l, l, plan->R, plan->Dbits, plan->Dtbits, plan->dt_words, plan->r, plan->rp,
        w.ssq + kSsqBlocks, (float)(1.0 / sqrt((double)l)));
    BSRHT_CO_LAUNCH_CHECK();
  }
  // 2. Cholesky factor of Omega Y (symmetrised)
  BSRHT_CO_TRY(sketch(w.Y, l, l, w.B));
  sym_f64_kernel<<<(unsigned)((l * l + 255) / 256), 256, 0, s>>>(w.B, l, l, w.Bs, l);
  BSRHT_CO_LAUNCH_CHECK();
  BSRHT_CO_TRY(scale_cols_f64(w.Bs, l, l, l, l, nullptr, w.Mf, l, s));
  BSRHT_CO_TRY(cholesky_upper(w.Mf, l, l, (double)l * kU64, w.flag, w.chol_state, s));
  int32_t hf = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hf, w.flag, sizeof(hf)));
  int64_t lz = l, ldz = l;  // columns of Z and its leading dimension
  if (hf == 0) {
    // 3. Z = Y C^{-1}
    BSRHT_CO_TRY(trinv_upper(w.Mf, l, l, w.Cinv, l, s));
    GemmDesc d;
    d.M = n; d.N = l; d.K = l;
    d.sai = l; d.sak = 1;
    d.sbk = l; d.sbj = 1;
    d.ldc = l;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, w.Y, w.Cinv, w.Z, s));
  } else {
    // Remark 3.1: B = V Lam V^T, keep Lam_i > l u Lam_max, Z = Y V_+ Lam_+^{-1/2}.
    // The eigenvectors come from a preconditioned problem when possible: for
    // c just above B's rounding-level negative eigenvalues, B + c I = C^T C
    // (Cholesky), and the right singular vectors of the triangular C are B's
    // eigenvectors; the one-sided Jacobi converges on C's columns in far
    // fewer sweeps than on B's.  c = ||B||_F 2^-24, then 16x, then 256x; if
    // none gives a factor, the Jacobi runs on B with rotation accumulation.
    // The signed eigenvalues are taken from B itself below either way.
    bool pre = false;
    ssq_partial_kernel<double><<<kSsqBlocks, 256, 0, s>>>(w.Bs, l, l, l, w.ssq);
    shift_of_kernel<<<1, 64, 0, s>>>(w.ssq, 1.0, w.ssq + kSsqBlocks);  // ||B||_F
    BSRHT_CO_LAUNCH_CHECK();
    for (int attempt = 0; attempt < 3 && !pre; ++attempt) {
      BSRHT_CO_TRY(scale_cols_f64(w.Bs, l, l, l, l, nullptr, w.Mf, l, s));
      add_diag_dev_kernel<<<(unsigned)((l + 255) / 256), 256, 0, s>>>(
          w.Mf, l, l, w.ssq + kSsqBlocks, kU32 * (double)(1 << (4 * attempt)));
      BSRHT_CO_LAUNCH_CHECK();
      BSRHT_CO_TRY(cholesky_upper(w.Mf, l, l, (double)l * kU64, w.flag + 2, w.chol_state, s));
      int32_t hc = 0;
      BSRHT_CO_TRY(co_await readback(ctx, &hc, w.flag + 2, sizeof(hc)));
      pre = hc == 0;
    }
    if (pre)
      BSRHT_CO_TRY(co_await small_svd_task(ctx, w.fb, w.Mf, l, l, false, info));
    else
      BSRHT_CO_TRY(co_await small_svd_task(ctx, w.fb, w.Bs, l, l, true, info));
    const int64_t nce = svd_pad(l);
    {
      // lambda_j = v_j^T (B v_j): W = B V into Cinv (unused on this path)
      GemmDesc d;
      d.M = l; d.N = l; d.K = l;
      d.sai = l; d.sak = 1;
      d.sbk = nce; d.sbj = 1;
      d.ldc = l;
      BSRHT_CO_TRY(gemm_f64(d, w.Bs, w.fb.Vs, w.Cinv, s));
      col_dots_kernel<<<(unsigned)((l + 3) / 4), 256, 0, s>>>(w.fb.Vs, nce, w.Cinv, l, l, w.lam);
      BSRHT_CO_LAUNCH_CHECK();
    }
    std::vector<double> lam((size_t)l);
    if (co_await readback(ctx, lam.data(), w.lam, sizeof(double) * (size_t)l) != BSRHT_OK)
      co_return BSRHT_EDEVICE;
    double lmax = 0.0;
    for (double x : lam) lmax = std::max(lmax, x);
    // kept columns in Jacobi order (descending |lambda|): the host decides
    // which (it sizes the products below); the arithmetic stays on the device
    std::vector<int32_t> idx;
    for (int64_t i = 0; i < l; ++i)
      if (lam[(size_t)i] > (double)l * kU64 * lmax && lam[(size_t)i] > 0.0)
        idx.push_back((int32_t)i);
    if (idx.empty()) co_return BSRHT_EDEVICE;
    lz = (int64_t)idx.size();
    // Z (n x lz) and Mf get a leading dimension rounded up to 4 elements,
    // which the large-tile GEMM kernel needs for its 16-byte loads.
    ldz = (lz + 3) & ~int64_t(3);
    // Mf = V_+ Lam_+^{-1/2} (l x lz, leading dimension ldz, zero padded)
    if (co_await upload(ctx, w.kidx, idx.data(), sizeof(int32_t) * (size_t)lz) != BSRHT_OK)
      co_return BSRHT_EDEVICE;
    inv_sqrt_kernel<<<(unsigned)((lz + 255) / 256), 256, 0, s>>>(w.lam, w.kidx, lz, w.fb.inv);
    gather_scale_cols_kernel<<<(unsigned)((l * ldz + 255) / 256), 256, 0, s>>>(
        w.fb.Vs, l, nce, w.kidx, w.fb.inv, lz, w.Mf, ldz);
    BSRHT_CO_LAUNCH_CHECK();
    GemmDesc d;
    d.M = n; d.N = lz; d.K = l;
    d.sai = l; d.sak = 1;
    d.sbk = ldz; d.sbj = 1;
    d.ldc = ldz;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, w.Y, w.Mf, w.Z, s));
    or_info_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_CHOL_FALLBACK);
    BSRHT_CO_LAUNCH_CHECK();
  }
  // 4. R-factor of Z with its columns in descending order of norm:
  // Z P = Q R, P^T Z^T Z P = R^T R.  The order makes R's rows graded, and the
  // one-sided Jacobi on R's rows then ends in fewer sweeps (a model of this
  // problem: 13 -> 11 at l = 512); the SVD of Z P is that of Z with the rows
  // of the right factor permuted, which step 6 undoes.
  const int gsz = gram_splits(n, lz);
  BSRHT_CO_TRY(gram_f64(w.Z, n, lz, ldz, 1, w.Gz, lz, w.gram_part, gsz, s));
  if (lz > kMaxOrderN) co_return BSRHT_EUNSUPPORTED;
  desc_diag_order_kernel<<<(unsigned)((lz + 255) / 256), 256, 0, s>>>(w.Gz, lz, lz, w.zperm);
  permute_sym_kernel<<<(unsigned)((lz * lz + 255) / 256), 256, 0, s>>>(w.Gz, lz, lz, w.zperm,
                                                                          w.Bs, lz);
  BSRHT_CO_LAUNCH_CHECK();
  BSRHT_CO_TRY(scale_cols_f64(w.Bs, lz, lz, lz, lz, nullptr, w.Gz, lz, s));
  BSRHT_CO_TRY(cholesky_upper(w.Gz, lz, lz, 1e-15 * (double)lz, w.flag + 1, w.chol_state, s));
  int32_t hz = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hz, w.flag + 1, sizeof(hz)));
  // 5. SVD of R (or the eigen decomposition of P^T Z^T Z P when R is singular)
  const double *Rsrc = hz == 0 ? w.Gz : w.Bs;
  BSRHT_CO_TRY(co_await small_svd_task(ctx, w.sv, Rsrc, lz, lz, hz != 0, info));
  if (hz != 0) {
    sqrt_clamp_kernel<<<(unsigned)((lz + 255) / 256), 256, 0, s>>>(w.sv.S, lz);
    BSRHT_CO_LAUNCH_CHECK();
  }
  // 6. U = Z P Vt_k St_k^{-1}; lambda = St_k^2
  finish_sigma_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(
      w.sv.S, lz, k, sqrt((double)lz * kU64), 2, w.sv.inv, lambda, info);
  BSRHT_CO_LAUNCH_CHECK();
  const int64_t keep = std::min(k, lz);
  const int64_t nce = svd_pad(lz);
  scale_cols_unpermute_kernel<<<(unsigned)((lz * k + 255) / 256), 256, 0, s>>>(
      w.sv.Vs, lz, nce, w.zperm, w.sv.inv, keep, k, w.Mk, k);
  BSRHT_CO_LAUNCH_CHECK();
  GemmDesc d;
  d.M = n; d.N = k; d.K = lz;
  d.sai = ldz; d.sak = 1;
  d.sbk = k; d.sbj = 1;
  d.ldc = k;
  BSRHT_CO_TRY(gemm_f64f64_f32(d, w.Z, w.Mk, U, s));
  if (shifted) {
    unshift_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(lambda, k, w.ssq + kSsqBlocks);
    BSRHT_CO_LAUNCH_CHECK();
  }
  co_return BSRHT_OK;
}

}  // namespace bsrht

extern "C" {

static int nystrom_blocking(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k, float *U,
                            double *lambda, int32_t *info, void *ws, size_t ws_bytes,
                            void *stream, bool shifted) {
  if (!plan || !A || !U || !lambda || !info || k < 1 || lda < plan->n) return BSRHT_EINVAL;
  if (ws_bytes < nystrom_workspace(plan, k) || !ws) return BSRHT_ENOMEM;
  DevCtx ctx;
  ctx.s = (hipStream_t)stream;
  return run_blocking(nystrom_task(ctx, plan, A, lda, k, U, lambda, info, ws, ws_bytes, shifted));
}

int nystrom(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k, float *U, double *lambda,
            int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return nystrom_blocking(plan, A, lda, k, U, lambda, info, ws, ws_bytes, stream, false);
}

int nystrom_shifted(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k, float *U,
                    double *lambda, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return nystrom_blocking(plan, A, lda, k, U, lambda, info, ws, ws_bytes, stream, true);
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Non-blocking forms: the same coroutines with an asynchronous context (one
// event, pinned staging), advanced by bsrht_task_poll / bsrht_task_wait.

struct bsrht_task_s {
  bsrht::DevCtx ctx;  // the coroutine refers to it: a task never moves
  std::optional<bsrht::Task> task;
  int status = BSRHT_OK;
  bool finished = false;
};

namespace {

constexpr size_t kTaskStagingHalf = 64 * 1024;  // pinned bytes per direction

int task_open(void *stream, bsrht_task_s **out) {
  auto *t = new (std::nothrow) bsrht_task_s;
  if (!t) return BSRHT_EDEVICE;
  t->ctx.s = (hipStream_t)stream;
  t->ctx.blocking = false;
  void *pin = nullptr;
  if (hipEventCreateWithFlags(&t->ctx.ev, hipEventDisableTiming) != hipSuccess) {
    delete t;
    return BSRHT_EDEVICE;
  }
  if (hipHostMalloc(&pin, 2 * kTaskStagingHalf, hipHostMallocDefault) != hipSuccess) {
    (void)hipEventDestroy(t->ctx.ev);
    delete t;
    return BSRHT_EDEVICE;
  }
  t->ctx.pinned = static_cast<char *>(pin);
  t->ctx.half_bytes = kTaskStagingHalf;
  *out = t;
  return BSRHT_OK;
}

// Resumes the task while the event it waits on has completed; 1 once it has
// finished (status set), 0 while the device is still busy.
int task_advance(bsrht_task_s *t) {
  while (!t->finished) {
    if (t->task->done()) {
      t->status = t->task->status();
      t->finished = true;
      break;
    }
    const hipError_t q = hipEventQuery(t->ctx.ev);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
      t->status = BSRHT_EDEVICE;
      t->finished = true;
      break;
    }
    t->ctx.resume_point.resume();
  }
  return 1;
}

int task_start(bsrht_task_s *t, bsrht::Task task, bsrht_task_t *out) {
  t->task.emplace(std::move(task));
  t->task->start();  // queues work up to the first readback
  (void)task_advance(t);
  *out = t;
  return BSRHT_OK;
}

}  // namespace

extern "C" {

int rsvd_start(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, int64_t k, float *U,
               double *S, float *V, int32_t *info, void *ws, size_t ws_bytes, void *stream,
               bsrht_task_t *task) {
  if (!task) return BSRHT_EINVAL;
  *task = nullptr;
  if (!plan || !A || !U || !S || !V || !info || m < 1 || k < 1 || lda < m) return BSRHT_EINVAL;
  if (ws_bytes < rsvd_workspace(plan, m, k) || !ws) return BSRHT_ENOMEM;
  bsrht_task_s *t = nullptr;
  BSRHT_TRY(task_open(stream, &t));
  return task_start(t, rsvd_task(t->ctx, plan, A, m, lda, k, U, S, V, info, ws, ws_bytes), task);
}

static int nystrom_start_impl(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k,
                              float *U, double *lambda, int32_t *info, void *ws,
                              size_t ws_bytes, void *stream, bool shifted, bsrht_task_t *task) {
  if (!task) return BSRHT_EINVAL;
  *task = nullptr;
  if (!plan || !A || !U || !lambda || !info || k < 1 || lda < plan->n) return BSRHT_EINVAL;
  if (ws_bytes < nystrom_workspace(plan, k) || !ws) return BSRHT_ENOMEM;
  bsrht_task_s *t = nullptr;
  BSRHT_TRY(task_open(stream, &t));
  return task_start(
      t, nystrom_task(t->ctx, plan, A, lda, k, U, lambda, info, ws, ws_bytes, shifted), task);
}

int nystrom_start(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k, float *U,
                  double *lambda, int32_t *info, void *ws, size_t ws_bytes, void *stream,
                  bsrht_task_t *task) {
  return nystrom_start_impl(plan, A, lda, k, U, lambda, info, ws, ws_bytes, stream, false, task);
}

int nystrom_shifted_start(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k, float *U,
                          double *lambda, int32_t *info, void *ws, size_t ws_bytes,
                          void *stream, bsrht_task_t *task) {
  return nystrom_start_impl(plan, A, lda, k, U, lambda, info, ws, ws_bytes, stream, true, task);
}

int bsrht_task_poll(bsrht_task_t task, int *status) {
  if (!task || !status) return BSRHT_EINVAL;
  if (!task_advance(task)) return 0;
  *status = task->status;
  return 1;
}

int bsrht_task_wait(bsrht_task_t task) {
  if (!task) return BSRHT_EINVAL;
  while (!task_advance(task)) {
    if (hipEventSynchronize(task->ctx.ev) != hipSuccess) {
      task->status = BSRHT_EDEVICE;
      task->finished = true;
    }
  }
  return task->status;
}

int bsrht_task_destroy(bsrht_task_t task) {
  if (!task) return BSRHT_EINVAL;
  (void)bsrht_task_wait(task);
  int st = BSRHT_OK;
  if (hipHostFree(task->ctx.pinned) != hipSuccess) st = BSRHT_EDEVICE;
  if (hipEventDestroy(task->ctx.ev) != hipSuccess) st = BSRHT_EDEVICE;
  delete task;  // the coroutine frame goes with its Task
  return st;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Single-view randomized SVD (section 3.3, Algorithm 3) for an N1 x N2
// row-major A with four block SRHTs: Omega (l x N2) and Psi (s x N2) act on
// the rows of A from the right, Gamma (l x N1) and Phi (s x N1) on its columns.
//   1. X^T = Gamma A (l x N2), Y = A Omega^T (N1 x l), Z = (Phi A) Psi^T (s x s)
//   2. Q = orth(Y), P = orth(X).  Q is kept implicit, Q = Y F with F the
//      inverse Cholesky factor of the FP64 Gram Y^T Y (the randomized SVD
//      treats its tall factor Z the same way): only Phi Q = (Phi Y) F and
//      U = Y (F M) are needed.  P (N2 x l) is formed by Cholesky-QR2.  A rank
//      deficient sketch keeps the directions of its Gram's eigen split.
//   3. Phi Q (s x lq), Psi P (s x lp)
//   4. C = (Phi Q)^+ Z ((Psi P)^T)^+ through the normal equations: Phi and Psi
//      are embeddings of the orthonormal Q and P, so the Grams of Phi Q and
//      Psi P are well conditioned (singular values near 1); G^{-1} = F F^T with
//      F the inverse Cholesky factor, or the eigen pseudo-inverse if a pivot
//      fails
//   5. C = Ut St Vt^T by one-sided Jacobi (Vt accumulated), k leading terms
//   6. U = Q (C Vt_k St_k^{-1}) = Q Ut_k, S = St_k, V = P Vt_k
// A is read three times (two column sketches, one row sketch).
namespace bsrht {
namespace {

template <class A>
struct SvWs {
  float *Xt, *Y, *W, *Zs, *PhY, *P32, *PsP, *Mu32, *Vk32;
  void *apply_ws;
  size_t apply_bytes;
  double *G, *Gs, *F, *Fq, *Q1, *G2, *C2inv, *gram_part;
  double *PhQ, *Gc, *F1, *F2, *T1, *T2, *T3t, *T4t, *Ct, *Mv, *Mu;
  int32_t *flag;
  void *chol_state;
  void *xws;  // split BF16 planes of Mu (U = Y Mu on split-BF16 matrix cores)
  size_t xws_bytes;
  SvdBufs<A> qb, sv;
  void layout(A &a, const bsrht_plan_s *om, const bsrht_plan_s *ga, const bsrht_plan_s *ph,
              const bsrht_plan_s *ps, int64_t k) {
    const int64_t N1 = ga->n, N2 = om->n, l = om->l, s = ph->l;
    const int64_t l4 = (l + 3) & ~int64_t(3);
    Xt = a.template take<float>((size_t)(l * N2));
    Y = a.template take<float>((size_t)(N1 * l));
    W = a.template take<float>((size_t)(s * N2));
    Zs = a.template take<float>((size_t)(s * s));
    // The column sketches of Q and P have lq, lp <= l columns; the workspace
    // of a sketch is not monotonic in its column count, so take the maximum.
    size_t ab = std::max({apply_ws_bytes(ga, N2), apply_right_ws_bytes(om, N1),
                          apply_ws_bytes(ph, N2), apply_right_ws_bytes(ps, s)});
    for (int64_t c = 1; c <= l; ++c) ab = std::max(ab, apply_ws_bytes(ps, c));
    ab = std::max(ab, apply_ws_bytes(ph, l));
    apply_bytes = ab;
    apply_ws = a.template take<char>(apply_bytes);
    G = a.template take<double>((size_t)(l * l));
    Gs = a.template take<double>((size_t)(l * l));
    F = a.template take<double>((size_t)(l4 * l4));
    Fq = a.template take<double>((size_t)(l * l));
    Q1 = a.template take<double>((size_t)(N2 * l4));
    G2 = a.template take<double>((size_t)(l * l));
    C2inv = a.template take<double>((size_t)(l4 * l4));
    gram_part = a.template take<double>((size_t)std::max(
        {gram_partial_elems(N1, l), gram_partial_elems(N2, l), gram_partial_elems(s, l),
         (int64_t)1}));
    PhY = a.template take<float>((size_t)(s * l));
    P32 = a.template take<float>((size_t)(N2 * l4));
    PhQ = a.template take<double>((size_t)(s * l));
    PsP = a.template take<float>((size_t)(s * l));
    Gc = a.template take<double>((size_t)(l * l));
    F1 = a.template take<double>((size_t)(l * l));
    F2 = a.template take<double>((size_t)(l * l));
    T1 = a.template take<double>((size_t)(l * s));
    T2 = a.template take<double>((size_t)(l * s));
    T3t = a.template take<double>((size_t)(l * l));
    T4t = a.template take<double>((size_t)(l * l));
    Ct = a.template take<double>((size_t)(l * l));
    Mv = a.template take<double>((size_t)(l * k));
    Mu = a.template take<double>((size_t)(l * k));
    Mu32 = a.template take<float>((size_t)(l * k));
    Vk32 = a.template take<float>((size_t)(l * k));
    flag = a.template take<int32_t>(4);
    chol_state = a.template take<char>(cholesky_state_bytes());
    xws_bytes = gemm_bf16x_ws_bytes(k, l, 3);
    xws = a.template take<char>(xws_bytes);
    qb.take(a, svd_pad(l), l);
    sv.take(a, svd_pad(l), k);
  }
};

// F (n x nf, row-major, leading dimension nf) with F F^T = G^{-1} for the
// symmetric positive semi-definite n x n G (overwritten): F = C^{-1} for the
// Cholesky factor G = C^T C, or, when a pivot is <= tol * max(diag(G)),
// F = V_+ Lam_+^{-1/2} from G's eigen split with the eigenvalues above
// n u lambda_max (then F F^T = G^+ and *fell_back is set).
template <class A>
Task inv_factor_task(DevCtx &ctx, double *G, int64_t n, double tol, double *F, int64_t *nf,
                     bool *fell_back, SvWs<A> &w, int32_t *info) {
  hipStream_t s = ctx.s;
  BSRHT_CO_TRY(scale_cols_f64(G, n, n, n, n, nullptr, w.Gs, n, s));
  BSRHT_CO_TRY(cholesky_upper(G, n, n, tol, w.flag, w.chol_state, s));
  int32_t hf = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hf, w.flag, sizeof(hf)));
  *fell_back = hf != 0;
  if (hf == 0) {
    *nf = n;
    co_return trinv_upper(G, n, n, F, n, s);
  }
  BSRHT_CO_TRY(co_await small_svd_task(ctx, w.qb, w.Gs, n, n, true, info));
  std::vector<double> ev((size_t)n);
  if (co_await readback(ctx, ev.data(), w.qb.S, sizeof(double) * (size_t)n) != BSRHT_OK)
    co_return BSRHT_EDEVICE;
  int64_t keep = 0;
  for (int64_t i = 0; i < n; ++i)
    if (ev[(size_t)i] > (double)n * kU64 * ev[0] && ev[(size_t)i] > 0.0) ++keep;
  if (keep < 1) keep = 1;
  inv_sqrt_kernel<<<(unsigned)((keep + 255) / 256), 256, 0, s>>>(w.qb.S, nullptr, keep, w.qb.inv);
  BSRHT_CO_LAUNCH_CHECK();
  BSRHT_CO_TRY(scale_cols_f64(w.qb.Vs, n, keep, keep, svd_pad(n), w.qb.inv, F, keep, s));
  *nf = keep;
  co_return BSRHT_OK;
}

// Q32 (rows x lk, leading dimension ld4(lk)): an orthonormal basis of the
// columns of X (rows x l, X[r][c] = X[r*sr + c*sc]) by Cholesky-QR2 in FP64;
// a rank deficient X keeps the lk <= l directions of its Gram's eigen split.
// Leading dimensions are rounded up to 4 elements (ld4), which the
// large-tile GEMM kernel needs for its 16-byte loads.
template <class A>
Task orth_basis_task(DevCtx &ctx, const float *X, int64_t rows, int64_t l, int64_t sr,
                     int64_t sc, float *Q32, int64_t *lk_out, SvWs<A> &w, int32_t *info) {
  hipStream_t s = ctx.s;
  BSRHT_CO_TRY(gram_f32(X, rows, l, sr, sc, w.G, l, w.gram_part, gram_splits(rows, l), s));
  int64_t lk = l;
  bool fb = false;
  BSRHT_CO_TRY(
      co_await inv_factor_task(ctx, w.G, l, (double)l * kU64, w.F, &lk, &fb, w, info));
  const int64_t ldk = ld4(lk);
  if (ldk != lk) {  // F (l x lk) into a zero padded l x ldk copy in C2inv
    BSRHT_CO_TRY(scale_cols_f64(w.F, l, lk, ldk, lk, nullptr, w.C2inv, ldk, s));
    BSRHT_CO_TRY(scale_cols_f64(w.C2inv, l, ldk, ldk, ldk, nullptr, w.F, ldk, s));
  }
  {
    GemmDesc d;
    d.M = rows; d.N = ldk; d.K = l;
    d.sai = sr; d.sak = sc;
    d.sbk = ldk; d.sbj = 1;
    d.ldc = ldk;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, X, w.F, w.Q1, s));
  }
  if (fb) {
    or_info_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_QB_FALLBACK);
    BSRHT_CO_LAUNCH_CHECK();
  }
  // second pass: G2 = Q1^T Q1 = C2^T C2, Q = Q1 C2^{-1} (padding columns stay 0)
  BSRHT_CO_TRY(gram_f64(w.Q1, rows, lk, ldk, 1, w.G2, lk, w.gram_part, gram_splits(rows, lk), s));
  BSRHT_CO_TRY(cholesky_upper(w.G2, lk, lk, 1e-14, w.flag + 1, w.chol_state, s));
  int32_t hf2 = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hf2, w.flag + 1, sizeof(hf2)));
  if (hf2 != 0) {  // Q1 is orthonormal to O(eps kappa^2): should not happen
    debug_report(__FILE__, __LINE__, "second Cholesky-QR pass", BSRHT_EDEVICE);
    co_return BSRHT_EDEVICE;
  }
  BSRHT_CO_TRY(trinv_upper(w.G2, lk, lk, w.F, ldk, s));
  BSRHT_CO_TRY(scale_cols_f64(w.F, lk, lk, ldk, ldk, nullptr, w.C2inv, ldk, s));
  if (ldk > lk) BSRHT_CO_TRY(fill_f64(w.C2inv + lk * ldk, (ldk - lk) * ldk, 0.0, s));
  GemmDesc d;
  d.M = rows; d.N = ldk; d.K = ldk;
  d.sai = ldk; d.sak = 1;
  d.sbk = ldk; d.sbj = 1;
  d.ldc = ldk;
  BSRHT_CO_TRY(gemm_f64f64_f32(d, w.Q1, w.C2inv, Q32, s));
  *lk_out = lk;
  co_return BSRHT_OK;
}

int sketch_cols(const bsrht_plan_s *pl, const float *X, int64_t m, int64_t ldx, float *Y,
                int64_t ldy, void *ws, size_t ws_bytes, hipStream_t s) {
  if (pl->precision == BSRHT_SPLIT_BF16)
    return apply_split_bf16(pl, X, m, ldx, Y, ldy, ws, ws_bytes, s);
  return apply_fp32(pl, X, m, ldx, Y, ldy, ws, ws_bytes, s);
}

bool sv_shapes_ok(const bsrht_plan_s *om, const bsrht_plan_s *ga, const bsrht_plan_s *ph,
                  const bsrht_plan_s *ps) {
  return om && ga && ph && ps && om->n == ps->n && ga->n == ph->n && om->l == ga->l &&
         ph->l == ps->l && om->l <= ph->l;
}

}  // namespace
}  // namespace bsrht

extern "C" {

size_t rsvd_single_view_workspace(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi,
                                  bsrht_plan_t psi, int64_t k) {
  if (!sv_shapes_ok(omega, gamma, phi, psi) || k < 1) return 0;
  SizeOnly so;
  SvWs<SizeOnly> w;
  w.layout(so, omega, gamma, phi, psi, k);
  return align256(so.sz.used);
}

}  // extern "C"

namespace bsrht {
namespace {

// The argument checks of rsvd_single_view and rsvd_single_view_start.
int sv_args(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi, bsrht_plan_t psi,
            const float *A, int64_t lda, int64_t k, float *U, double *S, float *V,
            int32_t *info, void *ws, size_t ws_bytes) {
  if (!sv_shapes_ok(omega, gamma, phi, psi) || !A || !U || !S || !V || !info || k < 1 ||
      lda < omega->n)
    return BSRHT_EINVAL;
  const int64_t N1 = gamma->n, N2 = omega->n, l = omega->l;
  if (svd_pad(l) > 4096 || N1 > INT_MAX || N2 > INT_MAX) return BSRHT_EUNSUPPORTED;
  if (ws_bytes < rsvd_single_view_workspace(omega, gamma, phi, psi, k) || !ws)
    return BSRHT_ENOMEM;
  return BSRHT_OK;
}

// Algorithm 3 (argument checks done by the caller).
Task rsvd_single_view_task(DevCtx &ctx, const bsrht_plan_s *omega, const bsrht_plan_s *gamma,
                           const bsrht_plan_s *phi, const bsrht_plan_s *psi, const float *A,
                           int64_t lda, int64_t k, float *U, double *S, float *V,
                           int32_t *info, void *ws, size_t ws_bytes) {
  const int64_t N1 = gamma->n, N2 = omega->n, l = omega->l, s_ = phi->l;
  hipStream_t s = ctx.s;
  Carve cv(ws, ws_bytes);
  SvWs<Carve> w;
  w.layout(cv, omega, gamma, phi, psi, k);
  if (cv.overflow) co_return BSRHT_ENOMEM;
  zero_i32_kernel<<<1, 64, 0, s>>>(info, 1);
  BSRHT_CO_LAUNCH_CHECK();

  // 1. the three sketches
  BSRHT_CO_TRY(sketch_cols(gamma, A, N2, lda, w.Xt, N2, w.apply_ws, w.apply_bytes, s));
  BSRHT_CO_TRY(apply_right_fp32(omega, A, N1, lda, w.Y, l, w.apply_ws, w.apply_bytes, s));
  BSRHT_CO_TRY(sketch_cols(phi, A, N2, lda, w.W, N2, w.apply_ws, w.apply_bytes, s));
  BSRHT_CO_TRY(apply_right_fp32(psi, w.W, s_, N2, w.Zs, s_, w.apply_ws, w.apply_bytes, s));
  // 2. Q = Y Fq implicitly (N1 x lq), P = orth(X) = orth(Xt^T) (N2 x lp)
  int64_t lq = l, lp = l;
  {
    bool fbq = false;
    BSRHT_CO_TRY(gram_f32(w.Y, N1, l, l, 1, w.G, l, w.gram_part, gram_splits(N1, l), s));
    BSRHT_CO_TRY(co_await inv_factor_task(ctx, w.G, l, (double)l * kU64, w.Fq, &lq, &fbq, w,
                                       info));
    if (fbq) {
      or_info_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_QB_FALLBACK);
      BSRHT_CO_LAUNCH_CHECK();
    }
  }
  BSRHT_CO_TRY(co_await orth_basis_task(ctx, w.Xt, N2, l, 1, N2, w.P32, &lp, w, info));
  const int64_t ldp = ld4(lp);  // leading dimension of P32
  // 3. Phi Q = (Phi Y) Fq (s x lq, FP64), Psi P (s x lp)
  BSRHT_CO_TRY(sketch_cols(phi, w.Y, l, l, w.PhY, l, w.apply_ws, w.apply_bytes, s));
  {
    GemmDesc d;
    d.M = s_; d.N = lq; d.K = l;
    d.sai = l; d.sak = 1;
    d.sbk = lq; d.sbj = 1;
    d.ldc = lq;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, w.PhY, w.Fq, w.PhQ, s));
  }
  BSRHT_CO_TRY(sketch_cols(psi, w.P32, lp, ldp, w.PsP, lp, w.apply_ws, w.apply_bytes, s));
  // 4. C = (Phi Q)^+ Z ((Psi P)^T)^+, computed as C^T (lp x lq) in Ct
  int64_t nf1 = lq, nf2 = lp;
  bool fb1 = false, fb2 = false;
  BSRHT_CO_TRY(gram_f64(w.PhQ, s_, lq, lq, 1, w.Gc, lq, w.gram_part, gram_splits(s_, lq), s));
  BSRHT_CO_TRY(co_await inv_factor_task(ctx, w.Gc, lq, (double)lq * kU64, w.F1, &nf1, &fb1, w,
                                       info));
  BSRHT_CO_TRY(gram_f32(w.PsP, s_, lp, lp, 1, w.Gc, lp, w.gram_part, gram_splits(s_, lp), s));
  BSRHT_CO_TRY(co_await inv_factor_task(ctx, w.Gc, lp, (double)lp * kU64, w.F2, &nf2, &fb2, w,
                                       info));
  if (fb1 || fb2) {
    or_info_kernel<<<1, 1, 0, s>>>(info, BSRHT_INFO_CHOL_FALLBACK);
    BSRHT_CO_LAUNCH_CHECK();
  }
  {
    GemmDesc d;  // T1^T = Z^T (Phi Q)  (s x lq), in T1
    d.M = s_; d.N = lq; d.K = s_;
    d.sai = 1; d.sak = s_;
    d.sbk = lq; d.sbj = 1;
    d.ldc = lq;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, w.Zs, w.PhQ, w.T1, s));
  }
  {
    GemmDesc d;  // T2 = F1^T T1  (nf1 x s), T1[kk][j] read from T1^T
    d.M = nf1; d.N = s_; d.K = lq;
    d.sai = 1; d.sak = nf1;
    d.sbk = 1; d.sbj = lq;
    d.ldc = s_;
    BSRHT_CO_TRY(gemm_f64(d, w.F1, w.T1, w.T2, s));
  }
  {
    GemmDesc d;  // C1 = F1 T2 = (Phi Q)^+ Z  (lq x s), into T1
    d.M = lq; d.N = s_; d.K = nf1;
    d.sai = nf1; d.sak = 1;
    d.sbk = s_; d.sbj = 1;
    d.ldc = s_;
    BSRHT_CO_TRY(gemm_f64(d, w.F1, w.T2, w.T1, s));
  }
  {
    GemmDesc d;  // T3t = (Psi P)^T C1^T  (lp x lq)
    d.M = lp; d.N = lq; d.K = s_;
    d.sai = 1; d.sak = lp;
    d.sbk = 1; d.sbj = s_;
    d.ldc = lq;
    BSRHT_CO_TRY(gemm_f32f64_f64(d, w.PsP, w.T1, w.T3t, s));
  }
  {
    GemmDesc d;  // T4t = F2^T T3t  (nf2 x lq)
    d.M = nf2; d.N = lq; d.K = lp;
    d.sai = 1; d.sak = nf2;
    d.sbk = lq; d.sbj = 1;
    d.ldc = lq;
    BSRHT_CO_TRY(gemm_f64(d, w.F2, w.T3t, w.T4t, s));
  }
  {
    GemmDesc d;  // Ct = F2 T4t = C^T  (lp x lq)
    d.M = lp; d.N = lq; d.K = nf2;
    d.sai = nf2; d.sak = 1;
    d.sbk = lq; d.sbj = 1;
    d.ldc = lq;
    BSRHT_CO_TRY(gemm_f64(d, w.F2, w.T4t, w.Ct, s));
  }
  // 5. SVD of C (lq x lp), preconditioned: the Cholesky factor R of the FP64
  // Gram C^T C = R^T R has the singular values and right singular vectors of
  // C, and the one-sided Jacobi converges on R's columns in far fewer sweeps
  // than on C's.  If that Cholesky fails (C numerically rank deficient), the
  // Jacobi runs on C itself: the row-major lp x lq Ct is C in column-major
  // order, and the rotations (Vt) are accumulated.
  const int64_t L = svd_pad(std::max(lq, lp));
  int64_t ldv = L;  // leading dimension of the right singular vectors in sv.Vs
  BSRHT_CO_TRY(gram_f64(w.Ct, lq, lp, 1, lq, w.Gc, lp, w.gram_part, gram_splits(lq, lp), s));
  BSRHT_CO_TRY(cholesky_upper(w.Gc, lp, lp, (double)lp * kU64, w.flag + 2, w.chol_state, s));
  int32_t hc = 0;
  BSRHT_CO_TRY(co_await readback(ctx, &hc, w.flag + 2, sizeof(hc)));
  if (hc == 0) {
    BSRHT_CO_TRY(co_await small_svd_task(ctx, w.sv, w.Gc, lp, lp, false, info));
    ldv = svd_pad(lp);
  } else {
    BSRHT_CO_TRY(fill_f64(w.sv.X, L * L, 0.0, s));
    BSRHT_CO_TRY(scale_cols_f64(w.Ct, lp, lq, lq, lq, nullptr, w.sv.X, L, s));
    BSRHT_CO_TRY(jacobi_svd(w.sv.X, L, L, L, w.sv.V, w.sv.S, w.sv.Vs, L, w.sv.perm, w.sv.flags,
                         kMaxSweeps, info, s));
  }
  // 6. S = St_k, V = P Vt_k, U = Q (C Vt_k St_k^{-1})
  const int64_t avail = std::min(lq, lp);
  finish_sigma_kernel<<<(unsigned)((k + 255) / 256), 256, 0, s>>>(
      w.sv.S, avail, k, sqrt((double)L * kU64), 1, w.sv.inv, S, info);
  BSRHT_CO_LAUNCH_CHECK();
  const int64_t keep = std::min(k, avail);
  BSRHT_CO_TRY(scale_cols_f64_f32(w.sv.Vs, lp, keep, k, ldv, nullptr, w.Vk32, k, s));
  {
    GemmDesc d;
    d.M = N2; d.N = k; d.K = lp;
    d.sai = ldp; d.sak = 1;
    d.sbk = k; d.sbj = 1;
    d.ldc = k;
    BSRHT_CO_TRY(gemm_f32(d, w.P32, w.Vk32, V, s));
  }
  BSRHT_CO_TRY(scale_cols_f64(w.sv.Vs, lp, keep, k, ldv, w.sv.inv, w.Mv, k, s));
  {
    GemmDesc d;  // Mu = C Mv = Ct^T Mv  (lq x k)
    d.M = lq; d.N = k; d.K = lp;
    d.sai = 1; d.sak = lq;
    d.sbk = k; d.sbj = 1;
    d.ldc = k;
    BSRHT_CO_TRY(gemm_f64(d, w.Ct, w.Mv, w.Mu, s));
  }
  {
    GemmDesc d;  // Mq = Fq Mu  (l x k), in Mv: U = Q Mu = Y Mq
    d.M = l; d.N = k; d.K = lq;
    d.sai = lq; d.sak = 1;
    d.sbk = k; d.sbj = 1;
    d.ldc = k;
    BSRHT_CO_TRY(gemm_f64(d, w.Fq, w.Mu, w.Mv, s));
  }
  BSRHT_CO_TRY(scale_cols_f64_f32(w.Mv, l, k, k, k, nullptr, w.Mu32, k, s));
  // the tall product with FP32-level accuracy (six split-BF16 products)
  co_return tall_product(w.Y, l, w.Mu32, k, U, k, N1, k, l, 3, w.xws, w.xws_bytes, s);
}

}  // namespace
}  // namespace bsrht

extern "C" {

int rsvd_single_view(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi, bsrht_plan_t psi,
                     const float *A, int64_t lda, int64_t k, float *U, double *S, float *V,
                     int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  BSRHT_TRY(sv_args(omega, gamma, phi, psi, A, lda, k, U, S, V, info, ws, ws_bytes));
  DevCtx ctx;
  ctx.s = (hipStream_t)stream;
  return run_blocking(rsvd_single_view_task(ctx, omega, gamma, phi, psi, A, lda, k, U, S, V,
                                            info, ws, ws_bytes));
}

int rsvd_single_view_start(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi,
                           bsrht_plan_t psi, const float *A, int64_t lda, int64_t k, float *U,
                           double *S, float *V, int32_t *info, void *ws, size_t ws_bytes,
                           void *stream, bsrht_task_t *task) {
  if (!task) return BSRHT_EINVAL;
  *task = nullptr;
  BSRHT_TRY(sv_args(omega, gamma, phi, psi, A, lda, k, U, S, V, info, ws, ws_bytes));
  bsrht_task_s *t = nullptr;
  BSRHT_TRY(task_open(stream, &t));
  return task_start(t, rsvd_single_view_task(t->ctx, omega, gamma, phi, psi, A, lda, k, U, S, V,
                                             info, ws, ws_bytes),
                    task);
}

}  // extern "C"
