// Internal dense linear-algebra kernels (see dense.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace bsrht {

// C = alpha * A B + beta * C with A[i][k] = A[i*sai + k*sak] (M x K),
// B[k][j] = B[k*sbk + j*sbj] (K x N), C row-major with leading dimension ldc.
// splits > 1 writes FP64 partial products at C + s*split_stride (beta = 0).
struct GemmDesc {
  int64_t M = 0, N = 0, K = 0;
  int64_t sai = 0, sak = 0, sbk = 0, sbj = 0;
  int64_t ldc = 0;
  double alpha = 1.0, beta = 0.0;
  int splits = 1;
  int64_t split_stride = 0;
  bool upper_tiles = false;  // compute only workgroup tiles on or above the diagonal
};

int gemm_f32(const GemmDesc &d, const float *A, const float *B, float *C, hipStream_t s);
int gemm_f64(const GemmDesc &d, const double *A, const double *B, double *C, hipStream_t s);
int gemm_f32f64_f64(const GemmDesc &d, const float *A, const double *B, double *C,
                    hipStream_t s);
int gemm_f64f64_f32(const GemmDesc &d, const double *A, const double *B, float *C,
                    hipStream_t s);
int gemm_f32f32_f64(const GemmDesc &d, const float *A, const float *B, double *C,
                    hipStream_t s);

// C = A B (FP32 operands on the FP32 matrix cores) with the K range split
// into `splits` FP32-accumulated partials, stored as FP64 at
// partials + s*M*N (splits*M*N doubles) and summed in split order into C
// (row-major, d.ldc; alpha = 1, beta = 0).  splits <= 1 is gemm_f32.
int gemm_f32_splitk(const GemmDesc &d, const float *A, const float *B, float *C,
                    double *partials, int splits, hipStream_t s);

// C (M x N, ldc) = A (M x K, FP32, row-major, lda a multiple of 4, 16-byte
// aligned) times B (K x N, FP32, row stride ldb) on the BF16 matrix cores,
// both operands split into `parts` BF16 parts (2: three products, ~2^-16
// relative; 3: six products, the accuracy of an FP32 product).  ws: device
// scratch of gemm_bf16x_ws_bytes(N, K, parts) bytes for B's split planes.
int gemm_f32_bf16x(const float *A, int64_t lda, const float *B, int64_t ldb, float *C,
                   int64_t ldc, int64_t M, int64_t N, int64_t K, int parts, void *ws,
                   size_t ws_bytes, hipStream_t s);
size_t gemm_bf16x_ws_bytes(int64_t N, int64_t K, int parts);
bool gemm_bf16x_eligible(const float *A, int64_t lda);

// G = X^T X (K x K FP64) for X[r][c] = X[r*sr + c*sc], r < n, c < K; the row
// range is split into `splits` FP64 partials (K*K each, in `partials`)
// summed in split order.  gram_f32 of a tall X (n >= 16384, sc == 1) runs on
// the int8 matrix cores with exact digit products (FP64-level accuracy, at
// most `splits` partials) and uses G itself as scratch before writing it.
int gram_f32(const float *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
             int64_t ldg, double *partials, int splits, hipStream_t s);
int gram_f64(const double *X, int64_t n, int64_t K, int64_t sr, int64_t sc, double *G,
             int64_t ldg, double *partials, int splits, hipStream_t s);
int gram_splits(int64_t n, int64_t K);
// FP64 elements of split-K partials any Gram call with rows <= n (n fixed)
// and K <= Kmax may need.
int64_t gram_partial_elems(int64_t n, int64_t Kmax);

// In-place FP64 Cholesky of the symmetric G (upper triangle read): G = C^T C,
// C upper.  *info (device) = 0 on success, else the 1-based index of the first
// pivot <= tol * max(diag(G)).
// `state` is device scratch of cholesky_state_bytes() bytes.
int cholesky_upper(double *G, int64_t n, int64_t ldg, double tol, int32_t *info, void *state,
                   hipStream_t s);
size_t cholesky_state_bytes();
// n <= 2048.
int trinv_upper(const double *C, int64_t n, int64_t ldc, double *Ci, int64_t ldi, hipStream_t s);
int eye(double *M, int64_t n, int64_t ld, hipStream_t s);
int fill_f64(double *p, int64_t count, double value, hipStream_t s);

// Workgroups of a block-Jacobi launch at most (nc <= 4096, 16-column pairs),
// and the flag words a run needs: the noise floor (two words), then two
// slots per workgroup.
constexpr int kJacobiMaxGroups = 256;
constexpr int kJacobiFlagWords = 2 + 2 * kJacobiMaxGroups;

// One-sided block Jacobi on the columns of X (nr x nc, column-major, ldx),
// nc a multiple of 32, nc <= 4096, nr <= 4096: X is overwritten by
// X V = U Sigma; S (nc, descending) is written, and Us (row-major, ldu)
// receives in the same order either the normalised columns U (V == NULL:
// nr x nc, the left singular vectors of X) or, when V (nc * nc doubles,
// scratch) is given, the accumulated rotations (nc x nc: the right singular
// vectors; for symmetric X, eigenvectors that stay orthogonal to working
// precision).  perm (nc int32) and flags (kJacobiFlagWords uint, 8-byte
// aligned) are scratch; S and Us also serve as scratch until the run's last
// launches write them (S must not alias X, V or Us).  Pairs with a column
// norm at or below u ||X||_F (u = 2^-53) count as orthogonal, so
// rank-deficient inputs converge.  When max_sweeps sweeps still rotate,
// BSRHT_INFO_JACOBI_NOCONV is or-ed into *info (device, may be NULL).
// Synchronises the stream once per sweep.
int jacobi_svd(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
               double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
               int32_t *info, hipStream_t s);
// The same with the form of the block step forced: 1 = 16-column block pairs
// staged in LDS (at most 1024 rows, and V of at most 1024 rows), 2 =
// 32-column block pairs streamed from global memory (any row count), or 0 to
// pick as jacobi_svd does (1 when it applies).
int jacobi_svd_shape(double *X, int64_t nr, int64_t nc, int64_t ldx, double *V, double *S,
                     double *Us, int64_t ldu, int32_t *perm, unsigned int *flags, int max_sweeps,
                     int32_t *info, int form, hipStream_t s);

int transpose_f32_f64(const float *src, int64_t rows, int64_t cols, int64_t lds, double *dst,
                      int64_t ldd, hipStream_t s);
int transpose_f32(const float *src, int64_t rows, int64_t cols, int64_t lds, float *dst,
                  int64_t ldd, hipStream_t s);
int transpose_f64(const double *src, int64_t rows, int64_t cols, int64_t lds, double *dst,
                  int64_t ldd, hipStream_t s);

// dst[i][j] = src[i][j] * scale[j] for j < keep (scale NULL: 1), 0 for
// keep <= j < out.
int scale_cols_f64_f32(const double *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                       const double *scale, float *dst, int64_t ldd, hipStream_t s);
int scale_cols_f64(const double *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                   const double *scale, double *dst, int64_t ldd, hipStream_t s);
int scale_cols_f32(const float *src, int64_t rows, int64_t keep, int64_t out, int64_t lds,
                   const double *scale, float *dst, int64_t ldd, hipStream_t s);

}  // namespace bsrht
