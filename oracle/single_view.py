"""Single-view randomized SVD (section 3.3, Algorithm 3) in FP64.

Oracle side; test infrastructure.  All four sketching matrices are block
SRHTs of oracle.sketch, so every call takes the same four Plans the GPU
library is given.

For an N1 x N2 matrix A (the paper's m x n), with Omega (l x N2),
Gamma (l x N1), Phi (s x N1) and Psi (s x N2), l <= s:
    1. X = A^T Gamma^T = (Gamma A)^T            (N2 x l)
       Y = A Omega^T                             (N1 x l)
       Z = Phi A Psi^T                           (s x s)
    2. Q = orth(Y)   (a basis of range(A Omega^T), N1 x l)
       P = orth(X)   (a basis of range(A^T Gamma^T), N2 x l)
    3. Phi Q (s x l) and Psi P (s x l)
    4. C = (Phi Q)^+ Z ((Psi P)^T)^+              (l x l), least squares
    5. C = Ut St Vt^T (SVD), truncated to k
    6. A ~= (Q Ut_k) St_k (P Vt_k)^T
Readings.  Step 2 pairs Q with range(A Omega^T) and P with
range(A^T Gamma^T), as the definition of the two subspaces in section 3.3
does (the step's wording lists X before Y).  In step 4 the right factor must
be the pseudo-inverse of (Psi P)^T (s x l) for the product to be l x l; it is
the minimiser of ||Phi (A - Q C P^T) Psi^T||_F over C, the core problem
that defines the approximation in section 3.3.  Step 6 as printed lacks the
transpose on P Vt_k.

Every step is a plain library call: SVDs (LAPACK gesdd) for the range bases
and the core, least squares (gelsd), so the oracle shares no algorithm with
the GPU path (Cholesky-QR, normal equations on well-conditioned embeddings,
Jacobi).
"""

import numpy as np

from .sketch import sketch, sketch_right


def sketches(omega, gamma, phi, psi, A):
    """Step 1: X = (Gamma A)^T, Y = A Omega^T, Z = Phi A Psi^T."""
    A = np.asarray(A, dtype=np.float64)
    X = sketch(gamma, A).T
    Y = sketch_right(omega, A)
    Z = sketch_right(psi, sketch(phi, A))
    return X, Y, Z


def orth(M):
    """An orthonormal basis of range(M): the left singular vectors whose
    singular values exceed numpy's numerical-rank tolerance
    (max(shape) * eps * sigma_max).  For a full-rank M this spans the same
    space as a QR factor; for a rank-deficient sketch (two samples that give
    collinear rows, e.g. a repeated index when p = 1) it spans range(M) only,
    where a QR factor would add completion columns outside it."""
    U, sg, _ = np.linalg.svd(M, full_matrices=False)
    tol = max(M.shape) * np.finfo(np.float64).eps * sg[0]
    return U[:, sg > tol]


def bases(X, Y):
    """Step 2: Q = orth(Y), P = orth(X) (section 3.3 defines Q and P as
    orthonormal bases of range(A Omega^T) and range(A^T Gamma^T))."""
    return orth(Y), orth(X)


def core_matrix(PhQ, Z, PsP):
    """Step 4: C = (Phi Q)^+ Z ((Psi P)^T)^+ by two least-squares solves:
    C1 = argmin ||(Phi Q) C1 - Z||, then C = argmin ||C (Psi P)^T - C1||."""
    C1 = np.linalg.lstsq(PhQ, Z, rcond=None)[0]            # l x s
    return np.linalg.lstsq(PsP, C1.T, rcond=None)[0].T     # l x l


def single_view(omega, gamma, phi, psi, A, k):
    """Algorithm 3: returns (U N1 x k', S k', V N2 x k'), A ~= U diag(S) V^T,
    k' = min(k, rank of the core)."""
    A = np.asarray(A, dtype=np.float64)
    X, Y, Z = sketches(omega, gamma, phi, psi, A)
    Q, P = bases(X, Y)
    PhQ = sketch(phi, Q)                                   # step 3
    PsP = sketch(psi, P)
    C = core_matrix(PhQ, Z, PsP)
    Ut, St, VtT = np.linalg.svd(C)                         # step 5
    kk = min(int(k), St.shape[0])
    return Q @ Ut[:, :kk], St[:kk].copy(), P @ VtT.T[:, :kk]
