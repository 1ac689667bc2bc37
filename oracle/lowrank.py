"""Randomized SVD (Algorithm 1) and Nystrom (Algorithm 2) in FP64.

Oracle side; test infrastructure.  The sketch Omega is the block SRHT of
oracle.sketch, so every call takes the same Plan the GPU library is given.

Orientation.  The library sketches the n rows of a tall n x m matrix A, i.e.
it forms Omega A.  Algorithm 1 of section 3.1 is written for an m_p x n_p
matrix sketched from the right (Y = A_p Omega^T).  Running it on A_p = A^T
(m_p = m, n_p = n) gives, step by step,
    1. Y   = A_p Omega^T          = (Omega A)^T                 (m x l)
    2. Q   = qr(Y)                                             (m x l'), l' = min(l, m)
    3. Z   = Q^T A_p               = (A Q)^T                     (l' x n)
    4. P R = qr(Z^T)               = qr(A Q)                     (n x l'), (l' x l')
    5. R^T = Ut St Vt^T  (SVD), truncated to k
    6. A_p ~= (Q Ut_k) St_k (P Vt_k)^T
so  A ~= (P Vt_k) St_k (Q Ut_k)^T:  U = P Vt_k (n x k), S = St_k, V = Q Ut_k.

Nystrom (section 3.2, Algorithm 2) for a symmetric positive semi-definite
n x n A:
    1. Y = A Omega^T                                        (n x l)
    2. C = Cholesky factor of Omega Y, upper, Omega Y = C^T C
       (Omega Y is symmetrised first: it is symmetric in exact arithmetic)
    3. Z = Y C^{-1}  (backward substitution)
    4. R = R-factor of Z
    5. R = Ut St Vt^T (SVD), truncated to k
    6. U_hat = Z Vt_k St_k^{-1}
    7. A ~= U_hat St_k^2 U_hat^T
Step 6 as printed multiplies Y, not Z; that equals Q~ Ut_k (Z = Q~ R) only
when C = I.  Z Vt_k St_k^{-1} = Q~ Ut_k is the reading used here (the paper
itself names Q~ Ut_k as the stabler alternative).

Remark 3.1: Omega A Omega^T may be rank deficient and break the Cholesky
factorisation; a square root from an eigen/SVD decomposition is then used
instead.  Reading: the factorisation is declared failed when a pivot is
<= tau * max(diag(B)) with tau = l * u (u = 2**-53 here), and then
B = V Lam V^T, keep Lam_i > tau * Lam_max, Z = Y V_+ Lam_+^{-1/2}.
"""

import numpy as np
import scipy.linalg as sla

from .sketch import sketch

U_FP64 = 2.0 ** -53


def rsvd(plan, A, k):
    """Algorithm 1 on A^T; returns (U n x k', S k', V m x k'), k' = min(k, l').

    Householder QR (numpy/LAPACK) for steps 2 and 4 and an SVD for step 5, so
    the oracle shares no algorithm with the GPU path (Cholesky-QR + Jacobi).
    """
    A = np.asarray(A, dtype=np.float64)
    W = sketch(plan, A)                        # step 1: Y_p = (Omega A)^T = W^T
    Q, _ = np.linalg.qr(W.T, mode="reduced")   # step 2: m x l'
    Z = A @ Q                                  # step 3 (transposed): n x l'
    P, R = np.linalg.qr(Z, mode="reduced")     # step 4: Z = P R
    Ut, St, VtT = np.linalg.svd(R.T)           # step 5: R^T = Ut St Vt^T
    kk = min(int(k), St.shape[0])
    U = P @ VtT.T[:, :kk]                      # step 6, transposed back
    V = Q @ Ut[:, :kk]
    return U, St[:kk].copy(), V


def _cholesky_upper_or_none(B, tau):
    """Upper C with B = C^T C, or None when a pivot is <= tau * max(diag(B))."""
    thresh = tau * float(np.max(np.diag(B)))
    try:
        L = np.linalg.cholesky(B)
    except np.linalg.LinAlgError:
        return None
    if np.any(np.diag(L) ** 2 <= thresh):
        return None
    return L.T


def _nystrom_z(Y, B, l, u):
    """Steps 2-3 of Algorithm 2 from Y = A Omega^T and B = Omega Y: returns
    (Z, fallback_taken) with Z Z^T = Y B^+ Y^T (Remark 3.1 when needed)."""
    B = 0.5 * (B + B.T)                        # symmetric in exact arithmetic
    tau = l * u
    C = _cholesky_upper_or_none(B, tau)        # step 2
    if C is not None:
        Z = sla.solve_triangular(C, Y.T, trans="T", lower=False).T  # step 3
        return Z, False
    lam, V = np.linalg.eigh(B)                 # Remark 3.1 square root
    keep = lam > tau * lam.max()
    Z = Y @ (V[:, keep] / np.sqrt(lam[keep]))
    return Z, True


def nystrom_factor(plan, A, u=U_FP64):
    """Steps 1-3 of Algorithm 2: returns (Y, Z, fallback_taken).

    Z satisfies Z Z^T = Y (Omega Y)^+ Y^T (pseudo-inverse when Remark 3.1's
    fallback is taken).
    """
    A = np.asarray(A, dtype=np.float64)
    Y = sketch(plan, A.T).T                    # step 1: Y = A Omega^T
    B = sketch(plan, Y)                        # Omega Y
    Z, fb = _nystrom_z(Y, B, plan.l, u)
    return Y, Z, fb


def nystrom_from_sketch(Y, B, k, l, u=U_FP64):
    """Steps 2-6 of Algorithm 2 given the sketches Y = A Omega^T (n x l) and
    B = Omega Y (l x l), however they were computed; returns
    (U_hat n x k', lam k', fallback_taken)."""
    Y = np.asarray(Y, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Z, fb = _nystrom_z(Y, B, l, u)
    R = np.linalg.qr(Z, mode="r")              # step 4
    _, St, VtT = np.linalg.svd(R)              # step 5: R = Ut St Vt^T
    kk = min(int(k), St.shape[0])
    Uh = Z @ (VtT.T[:, :kk] / St[:kk])         # step 6 (read with Z, see above)
    return Uh, St[:kk] ** 2, fb


def nystrom(plan, A, k, u=U_FP64):
    """Algorithm 2; returns (U_hat n x k', lam k', fallback_taken)."""
    A = np.asarray(A, dtype=np.float64)
    Y = sketch(plan, A.T).T                    # step 1: Y = A Omega^T
    B = sketch(plan, Y)                        # Omega Y
    return nystrom_from_sketch(Y, B, k, plan.l, u)


def nystrom_shifted(plan, A, k, u=U_FP64):
    """Algorithm 2 on the shifted matrix A + nu I, the alternative to Remark
    3.1 that section 3.2 cites (Li et al., Algorithm 971, ACM TOMS 2017):
    the shift makes Omega (A + nu I) Omega^T positive definite, and nu is
    subtracted from the computed eigenvalues.  Reading: nu = sqrt(n) u ||Y||_F
    with u the unit roundoff of the sketch precision (2^-53 here, 2^-24 for
    an FP32 sketch), and since (A + nu I) Omega^T = Y + nu Omega^T only the
    sketch is shifted.  Returns (U_hat n x k', lam k', nu, fallback_taken) with
    lam = max(sigma^2 - nu, 0)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    Om = _omega_rows(plan)                     # Omega (l x n), closed form
    Y = sketch(plan, A.T).T                    # step 1: Y = A Omega^T
    nu = np.sqrt(n) * u * np.linalg.norm(Y)
    Ynu = Y + nu * Om.T                        # (A + nu I) Omega^T
    B = sketch(plan, Ynu)
    B = 0.5 * (B + B.T)
    tau = plan.l * u
    C = _cholesky_upper_or_none(B, tau)
    fb = C is None
    if not fb:
        Z = sla.solve_triangular(C, Ynu.T, trans="T", lower=False).T
    else:
        lam_b, Vb = np.linalg.eigh(B)
        keep = lam_b > tau * lam_b.max()
        Z = Ynu @ (Vb[:, keep] / np.sqrt(lam_b[keep]))
    R = np.linalg.qr(Z, mode="r")
    _, St, VtT = np.linalg.svd(R)
    kk = min(int(k), St.shape[0])
    Uh = Z @ (VtT.T[:, :kk] / St[:kk])
    return Uh, np.maximum(St[:kk] ** 2 - nu, 0.0), nu, fb


def _omega_rows(plan):
    """Omega (l x n) from eq. (2.3) entry by entry: the sketch of the
    identity, column block by column block (no size limit, O(l n log r))."""
    n = plan.n
    cols = []
    for c0 in range(0, n, 4096):
        c1 = min(n, c0 + 4096)
        E = np.zeros((n, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        cols.append(sketch(plan, E))
    return np.concatenate(cols, axis=1)

