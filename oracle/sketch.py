"""Block SRHT sketch Y = Omega @ A in FP64 (oracle side; test infrastructure).

Section 2 defines the SRHT Omega = sqrt(n/l) R H D (eq. (2.1)), with H the
Walsh-Hadamard matrix scaled by 1/sqrt(n) and written as a Kronecker power of
[[1, 1], [1, -1]]; and the block SRHT (eq. (2.3))

    Omega = [Omega^(1), ..., Omega^(p)],
    Omega^(i) = sqrt(r/l) Dt^(i) R H D^(i),   r = n/p,

applied blockwise as  Omega V = sum_i Omega^(i) V^(i)  (eq. (2.4)).

With 0-based indices and H_r[y, x] = (-1)^popcount(y & x) (the unscaled
Kronecker power in natural order), the scale sqrt(r/l) * (1/sqrt(r)) is
1/sqrt(l), so every entry is

    Omega[j, i*r + x] = Dt^(i)_j * (-1)^popcount(R_j & x) * D^(i)_x / sqrt(l).

A block size r that is not a power of two gives section 2's partial SRHT:
Omega^(i) is the first r columns of the SRHT of size rp (the next power of
two), i.e. the block is padded with rp - r zero rows; the closed form above
holds for x < r with R_j in [0, rp).

Two independent computations are provided and must agree:
  omega_explicit : the closed form above, entry by entry (small n only);
  sketch         : per block, signs -> radix-2 FWHT -> gather R -> signs,
                   blocks summed in order i = 0..p-1, then / sqrt(l).
"""

import numpy as np


def hadamard_sign(y, x):
    """(-1)^popcount(y & x): the entry H_r[y, x] of the unscaled Kronecker power."""
    par = np.bitwise_count(np.bitwise_and(y, x)) & 1
    return 1.0 - 2.0 * par.astype(np.float64)


def omega_explicit(plan):
    """Omega (l x n, float64) from the closed form of eq. (2.3); n <= 2**14."""
    if plan.n > (1 << 14):
        raise ValueError("explicit Omega is for small n only")
    l, r, p = plan.l, plan.r, plan.p
    x = np.arange(r, dtype=np.int64)
    blocks = []
    for i in range(p):
        h = hadamard_sign(plan.R[:, None], x[None, :])  # (l, r) rows R_j of H_r
        blocks.append(plan.Dt[i][:, None] * h * plan.D[i][None, :])
    return np.concatenate(blocks, axis=1) / np.sqrt(l)


def fwht_rows(B):
    """Unscaled Walsh-Hadamard transform along axis 0 (natural order).

    The Kronecker form of H (section 2) factors into log2(r) butterfly
    stages; stage h pairs rows x and x+h inside each group of 2h rows and
    maps (u, v) -> (u + v, u - v).  Returns H_r @ B for B of shape (r, ...).
    """
    B = np.array(B, dtype=np.float64, copy=True)
    r = B.shape[0]
    if r & (r - 1):
        raise ValueError("length must be a power of two")
    tail = B.shape[1:]
    h = 1
    while h < r:
        V = B.reshape((r // (2 * h), 2, h) + tail)
        u = V[:, 0].copy()
        v = V[:, 1].copy()
        V[:, 0] = u + v
        V[:, 1] = u - v
        h *= 2
    return B


def block_partial(plan, A, i):
    """Omega^(i) A^(i) without the final 1/sqrt(l): Dt^(i) R H_r D^(i) A^(i).

    A block of r rows that is not a power of two is padded with zero rows to
    rp (section 2's partial SRHT: the first r columns of H_rp)."""
    r, rp = plan.r, plan.rp
    Ai = np.asarray(A[i * r:(i + 1) * r], dtype=np.float64)
    B = np.zeros((rp,) + Ai.shape[1:])
    B[:r] = plan.D[i][:, None] * Ai      # D^(i): flip row signs; zero padding
    B = fwht_rows(B)                     # H_rp (unscaled)
    S = B[plan.R, :]                     # R: keep rows R_j, draw order
    return plan.Dt[i][:, None] * S       # Dt^(i): flip sample signs


def sketch(plan, A):
    """Y = Omega @ A (l x m, float64) via eq. (2.4), blocks summed in order."""
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != plan.n:
        raise ValueError("A must have n rows")
    Y = np.zeros((plan.l, A.shape[1]), dtype=np.float64)
    for i in range(plan.p):
        Y += block_partial(plan, A, i)
    return Y / np.sqrt(plan.l)


def sketch_parallel(plan, A, workers, col_chunk=256):
    """sketch(plan, A) with its per-block terms evaluated concurrently.

    The terms block_partial(plan, A[:, c0:c1], i) are computed on a pool of
    `workers` threads (the transform acts on each column separately, so a
    column slice gives exactly those columns of the term); each column slice
    then sums its blocks in order i = 0..p-1 and is scaled by 1/sqrt(l) once,
    as sketch() does, so the result is bitwise that of sketch()."""
    import concurrent.futures as cf

    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != plan.n:
        raise ValueError("A must have n rows")
    m = A.shape[1]
    slices = [(c0, min(m, c0 + col_chunk)) for c0 in range(0, m, col_chunk)] or [(0, 0)]
    tasks = [(i, c0, c1) for (c0, c1) in slices for i in range(plan.p)]
    with cf.ThreadPoolExecutor(max(1, int(workers))) as ex:
        parts = list(ex.map(lambda t: block_partial(plan, A[:, t[1]:t[2]], t[0]), tasks))
    Y = np.zeros((plan.l, m), dtype=np.float64)
    for (i, c0, c1), part in zip(tasks, parts):
        Y[:, c0:c1] += part                   # blocks of a slice arrive in order
    return Y / np.sqrt(plan.l)


def sketch_entry(plan, column, j):
    """One entry Y[j, c] from a single column of A (length n), eq. (2.3).

    Used to check a full-size sketch at sampled positions: it needs only the
    column and the tables, and costs O(n) per entry.
    """
    col = np.asarray(column, dtype=np.float64)
    r = plan.r
    x = np.arange(r, dtype=np.int64)
    h = hadamard_sign(np.int64(plan.R[j]), x)
    total = 0.0
    for i in range(plan.p):
        total += plan.Dt[i][j] * np.dot(h, plan.D[i] * col[i * r:(i + 1) * r])
    return total / np.sqrt(plan.l)


def sketch_right(plan, A):
    """Y = A @ Omega^T (m x l, float64): the sketch applied from the right, to
    the rows of an m x n A, as in Algorithm 1 (section 3.1).  By definition
    A Omega^T = (Omega A^T)^T, so this is eq. (2.4) on A^T, transposed."""
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[1] != plan.n:
        raise ValueError("A must have n columns")
    return sketch(plan, A.T).T


def sketch_right_entry(plan, row, j):
    """One entry Y[g, j] of A @ Omega^T from a single row of A (length n)."""
    return sketch_entry(plan, row, j)

