/*
 * bsrht.h - C ABI of the MI355X (gfx950) block SRHT library.
 *
 * Operation (Balabanov, Beaupere, Grigori, Lederer, "Block subsampled
 * randomized Hadamard transform for low-rank approximation on distributed
 * architectures", section 2, eq. (2.3)-(2.4)):
 *
 *   Omega = [Omega^(1) ... Omega^(p)],  Omega^(i) = sqrt(r/l) Dt^(i) R H D^(i),
 *   r = n/p,  H = Walsh-Hadamard matrix of order r scaled by 1/sqrt(r),
 *   D^(i) (r x r) and Dt^(i) (l x l) diagonal Rademacher signs, independent
 *   for every block, R an l x r uniform row sample shared by all blocks
 *   (with replacement by default), and
 *
 *   Y = Omega A = sum_i Omega^(i) A^(i)   for a tall n x m matrix A.
 *
 * Entry by entry, with H_r[y,x] = (-1)^popcount(y & x) (Kronecker power of
 * [[1,1],[1,-1]], natural order), Omega[j, i*r+x] =
 * Dt^(i)_j (-1)^popcount(R_j & x) D^(i)_x / sqrt(l).
 *
 * Conventions shared by every call
 *   - Matrices are row-major.  A leading dimension is the distance, in
 *     elements, between the starts of consecutive rows (>= the row length).
 *   - Every pointer named "device" is HIP device memory owned by the caller;
 *     the library never frees it.  The library allocates no device memory in
 *     bsrht_apply, rsvd or nystrom: all scratch comes from the caller's
 *     workspace, sized by the matching *_workspace query.
 *   - "stream" is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it and the call returns without waiting, except where a
 *     call says it synchronises.
 *   - Argument errors are detected before anything is enqueued and returned
 *     as a negative status; nothing is written in that case.  Numerical
 *     events are reported through the int32 `info` word (device memory),
 *     readable once the stream has completed.  No C++ exception crosses
 *     this interface.
 *   - A plan is immutable once built; several streams may apply the same
 *     plan concurrently, each with its own workspace and outputs.
 */
#ifndef BSRHT_H
#define BSRHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define BSRHT_OK 0
#define BSRHT_EINVAL (-1)       /* invalid argument (shape, pointer, mode) */
#define BSRHT_ENOMEM (-2)       /* caller-provided buffer too small        */
#define BSRHT_EDEVICE (-3)      /* a HIP call failed                        */
#define BSRHT_EUNSUPPORTED (-4) /* valid but not supported by this build    */

/* Sampling mode of R (section 2: the block SRHT samples with replacement;
 * the SRHT of eq. (2.1) allows either). */
#define BSRHT_WITH_REPLACEMENT 0
#define BSRHT_WITHOUT_REPLACEMENT 1

/* Arithmetic of the transform.  FP32: radix-2 butterflies in FP32.
 * SPLIT_BF16: Hadamard tiles on BF16 matrix cores with A split into a BF16
 * high and low part and FP32 accumulation. */
#define BSRHT_FP32 0
#define BSRHT_SPLIT_BF16 1

/* info word bits written by rsvd / nystrom. */
#define BSRHT_INFO_CHOL_FALLBACK 1 /* Remark 3.1 square-root fallback taken   */
#define BSRHT_INFO_RANK_CLAMPED 2  /* k reduced to the available rank          */
#define BSRHT_INFO_QB_FALLBACK 4   /* range basis built from an eigen split    */
#define BSRHT_INFO_JACOBI_NOCONV 8 /* Jacobi SVD stopped at its sweep limit    */

typedef struct bsrht_plan_s *bsrht_plan_t;

/* Library version string (static storage). */
const char *bsrht_version(void);

/* Text for a status code (static storage). */
const char *bsrht_strerror(int status);

/*
 * Device bytes needed for the random tables of a plan with these sizes
 * (R: l int32; D: p*rp bits; Dt: p*l bits; two gather lane orders, for the
 * column and the right-side kernels: l int32 each; each region 256-byte
 * aligned).
 * Returns 0 if the sizes are invalid (see bsrht_plan).
 */
size_t bsrht_plan_bytes(int64_t n, int64_t p, int64_t l);

/*
 * Build the tables of Omega (eq. (2.3)) from (seed, sampling) with the
 * library's counter-based generator (Philox4x64-10, SC'11):
 *   key = (seed, 0); one call gives 256 bits, bit b in word b/64, bit b%64;
 *   D^(i)_x  = bit (x%256) of philox((x/256, i, 2, 0)), bit 1 -> -1;
 *   Dt^(i)_j = bit (j%256) of philox((j/256, i, 3, 0)), bit 1 -> -1;
 *   R_j (with replacement)    = word0(philox((j, 0, 1, 0))) mod rp;
 *   R_j (without replacement) = partial Fisher-Yates over [0, rp) with
 *       t = j + floor(word0(philox((j,0,1,0))) * (rp - j) / 2^64).
 * rp is r rounded up to a power of two.  A block size r = n/p that is not a
 * power of two gives section 2's partial SRHT: Omega^(i) is the first r
 * columns of the rp-point SRHT, i.e. each block of A is treated as padded
 * with rp - r zero rows (never stored).  Such plans sketch with the FP32
 * kernels whatever their precision; bsrht_apply_right streams them with the
 * padded variant of its kernel when rp >= 256 (else it evaluates them
 * directly, O(n) per output) and bsrht_apply_batch rejects them.
 *
 * n, p, l     : Omega is l x n with p blocks of r = n/p columns.  Requires
 *               p >= 1, p | n, 1 <= l <= n, and l <= rp for sampling
 *               without replacement.  n < 2^31 and p*rp < 2^31.
 * seed        : 64-bit seed.
 * sampling    : BSRHT_WITH_REPLACEMENT or BSRHT_WITHOUT_REPLACEMENT.
 * precision   : BSRHT_FP32 or BSRHT_SPLIT_BF16 (used by bsrht_apply).
 * dev_mem     : device buffer of >= bsrht_plan_bytes(n,p,l) bytes, owned by
 *               the caller and kept alive for the plan's lifetime.
 * stream      : the tables are written on this stream; later calls on other
 *               streams must be ordered after it by the caller.  Sampling
 *               without replacement synchronises the stream once.
 * out         : receives the host-side plan handle.
 * Returns BSRHT_OK, BSRHT_EINVAL, BSRHT_ENOMEM (dev_bytes too small) or
 * BSRHT_EDEVICE.
 */
int bsrht_plan(int64_t n, int64_t p, int64_t l, uint64_t seed, int sampling,
               int precision, void *dev_mem, size_t dev_bytes, void *stream,
               bsrht_plan_t *out);

/* Free the host handle (not the caller's table memory). NULL is accepted. */
int bsrht_plan_destroy(bsrht_plan_t plan);

/* Sizes and mode recorded in a plan.  Any output pointer may be NULL. */
int bsrht_plan_info(bsrht_plan_t plan, int64_t *n, int64_t *p, int64_t *l,
                    int *sampling, int *precision);

/*
 * Copy the plan's tables to host memory (synchronises the plan's stream).
 * R     : host int32[l]            sample indices in [0, rp), draw order.
 * Dbits : host uint32[ceil(p*rp/32)]  bit (g%32) of word g/32 is the sign
 *                                  bit of D^(i)_x for g = i*rp + x
 *                                  (1 -> -1; g = the global row when r = rp).
 * Dtbits: host uint32[p*ceil(l/32)] bit (j%32) of word i*ceil(l/32) + j/32
 *                                  is the sign bit of Dt^(i)_j.
 * Any pointer may be NULL to skip that table.
 */
int bsrht_plan_export(bsrht_plan_t plan, int32_t *R, uint32_t *Dbits,
                      uint32_t *Dtbits);

/* Workspace bytes bsrht_apply needs for an n x m input (0 is possible). */
size_t bsrht_apply_workspace(bsrht_plan_t plan, int64_t m);

/*
 * Y = Omega A  (eq. (2.4)): every block's signs, Walsh-Hadamard transform,
 * row sample and output signs, summed over the p blocks on the device.  A
 * is read once from HBM; no block's full transform is stored.  The sum over
 * blocks is taken in a fixed order, so results are bitwise repeatable.
 *
 * A   : device float32, n x m, leading dimension lda >= m.
 * m   : number of columns, m >= 0 (m == 0 is a no-op).
 * Y   : device float32, l x m, leading dimension ldy >= m; must not overlap A.
 * ws  : device workspace of ws_bytes >= bsrht_apply_workspace(plan, m)
 *       (may be NULL when that is 0).
 */
int bsrht_apply(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda,
                float *Y, int64_t ldy, void *ws, size_t ws_bytes, void *stream);

/*
 * bsrht_apply without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and result as bsrht_apply
 * (bitwise), except that the row-split partials live in a scratch array of
 * BSRHT_NOALLOC_SCRATCH_BYTES that the library holds in every GPU's memory
 * for the life of the process (one per device, set up on the first call on
 * that device).  Allocates nothing: no hipMalloc, hipFree or allocating
 * library routine.  Every call on one GPU uses that GPU's array, and each
 * call overwrites all of the partials it reads, so calls that follow one
 * another on a GPU need no clearing; calls that overlap on one GPU (on
 * different streams without ordering) race on it and must not be made.
 * Returns BSRHT_ENOMEM, with nothing enqueued, when the call would need more
 * than BSRHT_NOALLOC_SCRATCH_BYTES (bsrht_apply_workspace(plan, m) above it);
 * otherwise as bsrht_apply.
 */
#define BSRHT_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int bsrht_apply_noalloc(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda,
                        float *Y, int64_t ldy, void *stream);

/* Workspace bytes bsrht_apply_right needs for an m x n input (0 is possible). */
size_t bsrht_apply_right_workspace(bsrht_plan_t plan, int64_t m);

/*
 * Y = A Omega^T: the same block SRHT applied from the right, to the rows of
 * A along their contiguous dimension (the sketch A Omega^T of Algorithm 1,
 * section 3.1, in the paper's own orientation; eq. (2.3)-(2.4) per row).
 * Equal to (Omega A^T)^T up to FP32 rounding; A is read once from HBM and no
 * block's full transform is stored.  The sum over blocks is taken in a fixed
 * order, so results are bitwise repeatable.  The butterflies run in FP32
 * whatever the plan's precision (the split-BF16 form is a bsrht_apply
 * variant only).  Blocks of r >= 256 columns, or padded to rp >= 256
 * (section 2's partial SRHT), take the streaming kernel; shorter blocks an
 * O(n) per output direct evaluation.
 *
 * A   : device float32, m x n (n = the plan's n), row-major, leading
 *       dimension lda >= n.
 * m   : number of rows, m >= 0 (m == 0 is a no-op).
 * Y   : device float32, m x l, row-major, leading dimension ldy >= l; must
 *       not overlap A.
 * ws  : device workspace of ws_bytes >= bsrht_apply_right_workspace(plan, m)
 *       (may be NULL when that is 0).
 * Returns BSRHT_OK, BSRHT_EINVAL (NULL pointers, lda < n, ldy < l, m > 2^31-1),
 * BSRHT_ENOMEM (workspace too small), BSRHT_EUNSUPPORTED (l*m > 2^40) or
 * BSRHT_EDEVICE; nothing is enqueued on an error.
 */
int bsrht_apply_right(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda,
                      float *Y, int64_t ldy, void *ws, size_t ws_bytes, void *stream);

/*
 * Several FP32 sketches (eq. (2.4) each, as bsrht_apply) in one persistent
 * launch: the workgroup tiles of all items run from a descriptor table in
 * device memory, followed by one launch that sums every item's row-split
 * partials.  For many small sketches this replaces two launches per item by
 * a fixed three-kernel sequence, which is captured into a HIP graph on the
 * first call for a given (device, table) and replayed by later calls with the
 * table rewritten (the descriptors are copied in, stream-ordered, before each
 * replay).
 *
 * items      : host array of count items; each item is exactly the argument
 *              set of a bsrht_apply call (ws of >= bsrht_apply_workspace(plan,
 *              m) bytes, m >= 1), and its Y is bitwise the result that call
 *              would give (same launch decomposition and summation order).
 *              Items must not share Y or ws.
 * count      : 0 .. BSRHT_BATCH_MAX (0 is a no-op).
 * table      : device memory of table_bytes >= bsrht_batch_table_bytes(),
 *              caller-owned, overwritten by each call.  Calls that use the
 *              same table must be ordered (one stream, or synchronised).
 * Errors     : BSRHT_EINVAL for bad arguments; BSRHT_EUNSUPPORTED for an item
 *              whose plan is split-BF16 or whose blocks are shorter than 64
 *              rows (use bsrht_apply); BSRHT_ENOMEM for a short workspace.
 *              Nothing is enqueued when an item is rejected.
 */
#define BSRHT_BATCH_MAX 64
typedef struct bsrht_apply_item_s {
  bsrht_plan_t plan;
  const float *A;
  int64_t m, lda;
  float *Y;
  int64_t ldy;
  void *ws;
  size_t ws_bytes;
} bsrht_apply_item_t;
size_t bsrht_batch_table_bytes(void);
int bsrht_apply_batch(const bsrht_apply_item_t *items, int count, void *table,
                      size_t table_bytes, void *stream);

/*
 * Releases what bsrht_apply_batch keeps for `table` on the current device:
 * its captured graph, the pinned staging of its descriptors and their copy
 * event (a later call with the table captures them again).  Every call that
 * used the table must have completed (the copy event is waited for; the
 * graph launch is not).  Returns BSRHT_OK (also when nothing was kept),
 * BSRHT_EINVAL for a NULL table, BSRHT_EDEVICE if a HIP release failed.
 */
int bsrht_batch_table_release(void *table);

/* Workspace bytes rsvd needs for an n x m input and target rank k. */
size_t rsvd_workspace(bsrht_plan_t plan, int64_t m, int64_t k);

/*
 * Randomized SVD (section 3.1, Algorithm 1) of the tall n x m matrix A,
 * sketched on its n side by the plan's Omega (Algorithm 1 run on A^T):
 *   W = Omega A; Q = orth(W^T) (m x l', l' = min(l, m); FP64 Cholesky-QR2,
 *   Q = I when l >= m); Z = A Q (matrix cores); Z = P Rz (FP64 Gram +
 *   Cholesky); Rz = Ut St Vt^T (FP64 one-sided Jacobi);
 *   U = P Ut_k = Z Vt_k St_k^{-1}, S = St_k, V = Q Vt_k,  A ~= U diag(S) V^T.
 *
 * A    : device float32 n x m, lda >= m.        k: 1 <= k.
 * U    : device float32 n x k (row-major, leading dimension k).
 * S    : device float64 k, descending.
 * V    : device float32 m x k (row-major, leading dimension k).
 * info : device int32; BSRHT_INFO_* bits.  When the available rank k' is
 *        below k, columns k'..k-1 of U, V and entries of S are zero and
 *        BSRHT_INFO_RANK_CLAMPED is set.
 * ws   : device workspace of >= rsvd_workspace(plan, m, k) bytes.
 */
int rsvd(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, int64_t k,
         float *U, double *S, float *V, int32_t *info, void *ws,
         size_t ws_bytes, void *stream);

/* Workspace bytes nystrom needs for target rank k (A is n x n). */
size_t nystrom_workspace(bsrht_plan_t plan, int64_t k);

/*
 * Nystrom approximation (section 3.2, Algorithm 2) of a symmetric positive
 * semi-definite n x n matrix A:
 *   Y = A Omega^T (= (Omega A)^T); B = Omega Y, symmetrised; B = C^T C (FP64
 *   Cholesky, C upper); Z = Y C^{-1}; Z = Q~ R (FP64 Gram + Cholesky);
 *   R = Ut St Vt^T (FP64 one-sided Jacobi); U = Z Vt_k St_k^{-1} (= Q~ Ut_k);
 *   lambda = St_k^2;  A ~= U diag(lambda) U^T.
 * Remark 3.1: when a Cholesky pivot of B is <= l * 2^-53 * max(diag(B)) (the
 * factorisation is FP64), B = V Lam V^T is used instead, keeping
 * Lam_i > l * 2^-53 * Lam_max and Z = Y V_+ Lam_+^{-1/2};
 * BSRHT_INFO_CHOL_FALLBACK is set.  rsvd and nystrom synchronise the stream
 * (to read this flag back) before returning; nystrom_start below does not.
 *
 * A      : device float32 n x n, lda >= n (only read through Omega).
 * U      : device float32 n x k (leading dimension k).
 * lambda : device float64 k, descending.
 * info   : device int32, BSRHT_INFO_* bits (as in rsvd).
 * ws     : device workspace of >= nystrom_workspace(plan, k) bytes.
 */
int nystrom(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k,
            float *U, double *lambda, int32_t *info, void *ws,
            size_t ws_bytes, void *stream);

/*
 * Shifted Nystrom: Algorithm 2 on A + nu I, the alternative to Remark 3.1's
 * fallback that section 3.2 cites (Li et al., Algorithm 971, ACM TOMS 2017).
 * The sketch is shifted, Y + nu Omega^T = (A + nu I) Omega^T, with
 * nu = sqrt(n) u_s ||Y||_F (u_s the unit roundoff of the sketch: 2^-24 for
 * FP32, 2^-17 for split-BF16; computed on the device), which makes
 * Omega (A + nu I) Omega^T positive definite whenever Omega has full row
 * rank; lambda = max(sigma^2 - nu, 0).  Arguments, workspace
 * (nystrom_workspace) and errors as for nystrom; the Remark 3.1 fallback
 * remains for a rank deficient Omega (info bit BSRHT_INFO_CHOL_FALLBACK).
 */
int nystrom_shifted(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k,
                    float *U, double *lambda, int32_t *info, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Non-blocking forms of rsvd, nystrom and nystrom_shifted (sections 3.1 and
 * 3.2, as above).  These algorithms read a few values back from the device
 * (Cholesky flags, the Jacobi sweep slots, the kept eigenvalues of Remark
 * 3.1), and the blocking forms synchronise their stream at those points.
 * The *_start forms take the blocking form's arguments plus `task`, check
 * them the same way (an error returns its code, enqueues nothing and sets
 * *task = NULL), queue the work up to the first readback on `stream` and
 * return at once with a task handle in *task.
 *
 * bsrht_task_poll(task, &status) advances the task as far as the device
 * allows without waiting: it returns 0 while the task waits on the device,
 * and 1 once all of the task's work has been queued, with *status set to
 * the blocking form's return value (BSRHT_EDEVICE if a HIP call failed).
 * The results are then ready in stream order: synchronise the stream, or
 * wait on an event recorded after the task, before reading them on the host.
 * bsrht_task_wait blocks until the task has been queued in full and returns
 * that status.  bsrht_task_destroy waits for an unfinished task and releases
 * it: the host handle, one HIP event and 128 KiB of pinned host staging,
 * which *_start allocates.  BSRHT_EINVAL for a NULL task.
 *
 * Until the task has finished, A, the outputs, info and the workspace belong
 * to it and the plan must stay valid.  A task is advanced by one thread at a
 * time; tasks on different streams, each with its own workspace, run
 * concurrently.  The arithmetic is that of the blocking forms: results are
 * bitwise the same.
 */
typedef struct bsrht_task_s *bsrht_task_t;
int rsvd_start(bsrht_plan_t plan, const float *A, int64_t m, int64_t lda, int64_t k,
               float *U, double *S, float *V, int32_t *info, void *ws,
               size_t ws_bytes, void *stream, bsrht_task_t *task);
int nystrom_start(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k,
                  float *U, double *lambda, int32_t *info, void *ws,
                  size_t ws_bytes, void *stream, bsrht_task_t *task);
int nystrom_shifted_start(bsrht_plan_t plan, const float *A, int64_t lda, int64_t k,
                          float *U, double *lambda, int32_t *info, void *ws,
                          size_t ws_bytes, void *stream, bsrht_task_t *task);
int bsrht_task_poll(bsrht_task_t task, int *status);
int bsrht_task_wait(bsrht_task_t task);
int bsrht_task_destroy(bsrht_task_t task);

/* Workspace bytes rsvd_single_view needs (0 for inconsistent plans or k < 1). */
size_t rsvd_single_view_workspace(bsrht_plan_t omega, bsrht_plan_t gamma,
                                  bsrht_plan_t phi, bsrht_plan_t psi, int64_t k);

/*
 * Single-view randomized SVD (section 3.3, Algorithm 3) of an N1 x N2 A with
 * four block SRHTs: omega (l x N2) and psi (s x N2) sketch the rows of A
 * from the right (bsrht_apply_right), gamma (l x N1) and phi (s x N1) its
 * columns (bsrht_apply), l <= s.  Forms X^T = Gamma A, Y = A Omega^T and the
 * core sketch Z = Phi A Psi^T, orthonormal bases Q of range(Y) and P of
 * range(X) (Cholesky-QR2 in FP64; a rank deficient sketch keeps the
 * directions of its Gram's eigen split above l*2^-53 relative and sets
 * BSRHT_INFO_QB_FALLBACK), the core C = (Phi Q)^+ Z ((Psi P)^T)^+ by FP64
 * normal equations (an eigen pseudo-inverse and BSRHT_INFO_CHOL_FALLBACK if
 * a Gram is singular), and the SVD C = Ut St Vt^T by one-sided Jacobi;
 * returns A ~= U diag(S) V^T with U = Q Ut_k, S = St_k, V = P Vt_k.  Entries
 * beyond the numerical rank of C are zero (BSRHT_INFO_RANK_CLAMPED).  A is
 * read three times.  Synchronises the stream where a Cholesky flag or the
 * eigenvalues of a fallback are needed (rsvd_single_view_start below does
 * not).
 *
 * omega, gamma, phi, psi: plans with omega->n == psi->n == N2,
 *     gamma->n == phi->n == N1, omega->l == gamma->l == l,
 *     phi->l == psi->l == s >= l (independent seeds); else BSRHT_EINVAL.
 *     The column sketches run in their plans' precision; the row sketches
 *     in FP32.
 * A   : device float32, N1 x N2 row-major, lda >= N2.
 * k   : target rank >= 1.
 * U   : device float32, N1 x k row-major;  S: device float64[k];
 * V   : device float32, N2 x k row-major;  info: device int32 (BSRHT_INFO_*).
 * ws  : device workspace of ws_bytes >= rsvd_single_view_workspace(...).
 * Returns BSRHT_OK, BSRHT_EINVAL, BSRHT_ENOMEM, BSRHT_EUNSUPPORTED (l > 4096
 * or N1, N2 >= 2^31) or BSRHT_EDEVICE.
 */
int rsvd_single_view(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi,
                     bsrht_plan_t psi, const float *A, int64_t lda, int64_t k,
                     float *U, double *S, float *V, int32_t *info, void *ws,
                     size_t ws_bytes, void *stream);

/*
 * Non-blocking form of rsvd_single_view (section 3.3, as above), under the
 * rules of the *_start forms before it: the same arguments plus `task`,
 * checked the same way, advanced by bsrht_task_poll / bsrht_task_wait and
 * released by bsrht_task_destroy; results bitwise those of the blocking form.
 */
int rsvd_single_view_start(bsrht_plan_t omega, bsrht_plan_t gamma, bsrht_plan_t phi,
                           bsrht_plan_t psi, const float *A, int64_t lda, int64_t k,
                           float *U, double *S, float *V, int32_t *info, void *ws,
                           size_t ws_bytes, void *stream, bsrht_task_t *task);

/*
 * Dense comparison sketches (section 4 compares the block SRHT with Gaussian
 * embeddings): Y = G A for an l x n Gaussian or Rademacher G, drawn from the
 * same Philox4x64-10 as the block SRHT tables, key (seed, 0):
 *   BSRHT_DENSE_GAUSSIAN   G[j][x] = z / sqrt(l), Box-Muller on word
 *       q = (x & 7) >> 1 of philox((x >> 3, j, 4, 0)): u1 from its low,
 *       u2 from its high 32 bits, u = (w + 1/2) 2^-32, z = sqrt(-2 ln u1) *
 *       cos(2 pi u2) for even x, * sin(2 pi u2) for odd x (FP64, rounded once
 *       to FP32);
 *   BSRHT_DENSE_RADEMACHER G[j][x] = +-1 / sqrt(l), bit (x & 255) of
 *       philox((x >> 8, j, 5, 0)), bit 1 -> -1.
 * G is materialised in the workspace (l x n FP32), then the product runs on
 * the FP32 matrix cores with the n-long contraction split into FP64 partials
 * summed in a fixed order (bitwise repeatable).
 *
 * A  : device float32, n x m, leading dimension lda >= m.
 * Y  : device float32, l x m, leading dimension ldy >= m.
 * ws : device workspace of ws_bytes >= bsrht_dense_workspace(n, l, m).
 * Returns BSRHT_OK, BSRHT_EINVAL (unknown kind, n or l < 1, m < 0, NULL
 * pointers, short leading dimensions), BSRHT_ENOMEM, BSRHT_EUNSUPPORTED
 * (a size >= 2^31) or BSRHT_EDEVICE; m == 0 is a no-op.
 */
#define BSRHT_DENSE_GAUSSIAN 0
#define BSRHT_DENSE_RADEMACHER 1
size_t bsrht_dense_workspace(int64_t n, int64_t l, int64_t m);
int bsrht_dense_sketch(int kind, uint64_t seed, int64_t n, int64_t l, const float *A,
                       int64_t m, int64_t lda, float *Y, int64_t ldy, void *ws,
                       size_t ws_bytes, void *stream);

/*
 * Instrumentation (not part of the computation).  bsrht_timing_enable(which)
 * makes the library record a pair of HIP events on the launching stream
 * around every launch of the selected kernel, until called again with 0;
 * bsrht_timing_read waits for the recorded events and returns the summed
 * kernel time in milliseconds and the number of launches since the enable.
 * Process-wide state, not thread-safe; for benchmarks.
 */
#define BSRHT_TIMING_OFF 0
#define BSRHT_TIMING_APPLY_FP32 1 /* the fused FP32 sketch kernel          */
#define BSRHT_TIMING_APPLY_BF16 2 /* the split-BF16 matrix-core kernel     */
#define BSRHT_TIMING_GEMM_AQ 3    /* Z = A Q of the randomized SVD          */
#define BSRHT_TIMING_STREAM 4     /* bsrht_stream_read                       */
#define BSRHT_TIMING_APPLY_RIGHT 5 /* the FP32 sketch kernel of bsrht_apply_right */
#define BSRHT_TIMING_DENSE_GEMM 6  /* the product of bsrht_dense_sketch (GEMM + reduce) */
int bsrht_timing_enable(int which);
int bsrht_timing_read(double *total_ms, int64_t *launches);
/*
 * The per-launch durations (milliseconds, in launch order) recorded since
 * bsrht_timing_enable: up to cap of them are written to ms (host); *count
 * receives the number of recorded launches.  Waits for the recorded events.
 * BSRHT_EINVAL for cap < 0 or ms == NULL with cap > 0.
 */
int bsrht_timing_samples(float *ms, int64_t cap, int64_t *count);

/*
 * Read-bandwidth reference (measurement, not part of the computation): reads
 * x[0 .. 4*floor(count/4)) once from device memory with 16-byte
 * non-temporal loads and writes one partial sum per workgroup to out
 * (BSRHT_STREAM_BLOCKS floats, device, caller-owned).  x must be 16-byte
 * aligned (else BSRHT_EINVAL).  Stream-ordered; timed under
 * BSRHT_TIMING_STREAM.  Its rate over a buffer larger than the 256 MB last
 * level cache is the read rate the sketch kernels' HBM traffic is compared
 * with.
 */
#define BSRHT_STREAM_BLOCKS 4096
int bsrht_stream_read(const float *x, int64_t count, float *out, void *stream);

/*
 * Releases every HIP object the library keeps for the life of the process:
 * the timing events and, for every table and device, the graphs, pinned
 * staging and events of bsrht_apply_batch.  Meant for the end of a program,
 * while the HIP runtime is still up (the Python binding calls it at
 * interpreter exit); no library call may be pending or follow except new
 * ones, which recreate what they need.  Returns BSRHT_OK or BSRHT_EDEVICE.
 */
int bsrht_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* BSRHT_H */
