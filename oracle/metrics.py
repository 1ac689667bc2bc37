"""Error measures used by the parity tests (oracle side; test infrastructure).

Section 3 measures a rank-k approximation against the best rank-k one in the
spectral, trace (nuclear) or Frobenius norm; the tail errors of [[A]]_k are
sigma_{k+1}, sum_{i>k} sigma_i and sqrt(sum_{i>k} sigma_i^2).  Figure 1
reports the relative trace error ||A - [[A]]_k^(Nyst)||_* / ||A||_*.
"""

import numpy as np


def rel_fro(X, X_ref):
    """||X - X_ref||_F / ||X_ref||_F in float64."""
    X = np.asarray(X, dtype=np.float64)
    X_ref = np.asarray(X_ref, dtype=np.float64)
    return float(np.linalg.norm(X - X_ref) / np.linalg.norm(X_ref))


def lowrank_fro_error(A, U, S, V, row_block=1 << 14):
    """||A - U diag(S) V^T||_F / ||A||_F, computed in float64 in row blocks."""
    A = np.asarray(A)
    U = np.asarray(U, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    num = 0.0
    den = 0.0
    SVt = S[:, None] * V.T
    for s in range(0, A.shape[0], row_block):
        Ab = np.asarray(A[s:s + row_block], dtype=np.float64)
        Eb = Ab - U[s:s + row_block] @ SVt
        num += float(np.sum(Eb * Eb))
        den += float(np.sum(Ab * Ab))
    return float(np.sqrt(num / den))


def trace_error(A, U, lam):
    """||A - U diag(lam) U^T||_* / ||A||_* with the nuclear norm as sum |eig|.

    A - U diag(lam) U^T is symmetric but, with a noisy sketch, not always
    positive semi-definite, so tr(A) - sum(lam) is not used.
    """
    A = np.asarray(A, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    E = A - (U * lam) @ U.T
    E = 0.5 * (E + E.T)
    num = float(np.sum(np.abs(np.linalg.eigvalsh(E))))
    den = float(np.sum(np.abs(np.linalg.eigvalsh(0.5 * (A + A.T)))))
    return num / den


def trace_error_structured(X, s, U, lam, shift=0.0):
    """||A - U diag(lam) U^T||_* / ||A||_* for A = X diag(s) X^T + shift I, with
    X (n x d) orthonormal, s >= 0 and shift >= 0, without forming A.

    E = A - U diag(lam) U^T maps every vector orthogonal to span[X, U] to
    shift times itself.  With B (n x q) any orthonormal basis containing
    span[X, U], the eigenvalues of E are those of B^T E B and shift with
    multiplicity n - q; ||A||_* = sum(s) + n shift.
    """
    X = np.asarray(X, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = X.shape[0]
    B, _ = np.linalg.qr(np.concatenate([X, U], axis=1), mode="reduced")
    XtB = X.T @ B
    UtB = U.T @ B
    E = (XtB.T * s) @ XtB - (UtB.T * lam) @ UtB + shift * np.eye(B.shape[1])
    ev = np.linalg.eigvalsh(0.5 * (E + E.T))
    num = float(np.sum(np.abs(ev))) + shift * (n - B.shape[1])
    return num / (float(np.sum(s)) + n * shift)


def optimal_fro_error(A, k):
    """||A - [[A]]_k||_F / ||A||_F from the singular values (section 3)."""
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(np.sqrt(np.sum(s[k:] ** 2) / np.sum(s ** 2)))


def optimal_trace_error(A, k):
    """||A - [[A]]_k||_* / ||A||_* for symmetric A (singular values = |eig|)."""
    s = np.sort(np.abs(np.linalg.eigvalsh(np.asarray(A, dtype=np.float64))))[::-1]
    return float(np.sum(s[k:]) / np.sum(s))


def ose_distortion(Omega, V):
    """max_i |sigma_i(Omega V)^2 - 1| for V with orthonormal columns (Def. 1.1)."""
    s = np.linalg.svd(np.asarray(Omega, dtype=np.float64) @ np.asarray(V, dtype=np.float64),
                      compute_uv=False)
    return float(np.max(np.abs(s ** 2 - 1.0)))
