"""Pins of the oracle's randomized SVD (Algorithm 1) and Nystrom (Algorithm 2).

Pinned against exact results (rank-k' inputs recovered to rounding), against
the optimal rank-k errors of section 3 computed with numpy's SVD / eigh, against
special cases that reduce to a plain truncated SVD / eigendecomposition
(orthogonal Omega, l >= m), and against the identities Algorithm 2 relies on.
"""
import numpy as np
import pytest

from oracle import rng, sketch, lowrank, metrics


def _lowrank(n, m, kk, seed):
    rs = np.random.default_rng(seed)
    X = rs.standard_normal((n, kk))
    W = rs.standard_normal((m, kk))
    return X @ W.T


def _decaying(n, m, seed, decay=lambda j: j ** -2.0):
    rs = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rs.standard_normal((n, m)))
    W, _ = np.linalg.qr(rs.standard_normal((m, m)))
    s = decay(np.arange(1, m + 1, dtype=np.float64))
    return (X * s) @ W.T


def _spd(n, d, seed, decay=lambda j: j ** -3.0):
    rs = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rs.standard_normal((n, d)))
    s = decay(np.arange(1, d + 1, dtype=np.float64))
    return (X * s) @ X.T


@pytest.mark.parametrize("p", [1, 4, 16])
def test_rsvd_exact_recovery(p):
    """P9: a rank-k' matrix with k' <= l - 10 is recovered to rounding."""
    n, m, l, kk = 1024, 96, 40, 30
    A = _lowrank(n, m, kk, 1)
    U, S, V = lowrank.rsvd(rng.Plan(n, p, l, 2), A, kk)
    assert metrics.lowrank_fro_error(A, U, S, V) < 1e-10


def test_rsvd_full_range_is_truncated_svd():
    """l >= m: range(Q) is all of R^m, so Algorithm 1 is the truncated SVD."""
    n, m, l, k = 512, 32, 64, 10
    A = _decaying(n, m, 3)
    U, S, V = lowrank.rsvd(rng.Plan(n, 4, l, 4), A, k)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(S, s[:k], rtol=1e-12)
    assert abs(metrics.lowrank_fro_error(A, U, S, V) - metrics.optimal_fro_error(A, k)) < 1e-12


def test_rsvd_near_optimal_and_bound():
    """P10/P11: error >= optimal, and within eq. (3.4)'s bound with d = l/4."""
    n, m, l, k = 4096, 256, 128, 50
    A = _decaying(n, m, 5)
    U, S, V = lowrank.rsvd(rng.Plan(n, 4, l, 0), A, k)
    err = metrics.lowrank_fro_error(A, U, S, V)
    opt = metrics.optimal_fro_error(A, k)
    d = l // 4
    tail_d = metrics.optimal_fro_error(A, d)
    assert opt <= err <= opt + 2.5 * tail_d
    assert err < 1.05 * opt
    assert np.allclose(np.linalg.norm(U, axis=0), 1.0, atol=1e-10)
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-10)
    assert np.allclose(V.T @ V, np.eye(k), atol=1e-10)


def test_rsvd_like_gaussian():
    """P12: block SRHT and Gaussian sketches give RSVD errors of the same size."""
    n, m, l, k = 2048, 128, 64, 20
    A = _decaying(n, m, 6, decay=lambda j: np.exp(-j / 8.0))
    eb = []
    eg = []
    rs = np.random.default_rng(7)
    for t in range(8):
        U, S, V = lowrank.rsvd(rng.Plan(n, 8, l, 100 + t), A, k)
        eb.append(metrics.lowrank_fro_error(A, U, S, V))
        G = rs.standard_normal((l, n))
        Q, _ = np.linalg.qr((G @ A).T)
        Z = A @ Q
        u, s, vt = np.linalg.svd(Z, full_matrices=False)
        eg.append(metrics.lowrank_fro_error(A, u[:, :k], s[:k], Q @ vt.T[:, :k]))
    assert np.mean(eb) < 1.3 * np.mean(eg) and np.mean(eg) < 1.3 * np.mean(eb)


def test_nystrom_orthogonal_omega_is_exact():
    """p = 1, l = r = n without replacement: Omega orthogonal, Nystrom = eigh truncation."""
    n, k = 256, 12
    A = _spd(n, n, 8, decay=lambda j: j ** -2.0)
    Uh, lam, fb = lowrank.nystrom(rng.Plan(n, 1, n, 9, rng.WITHOUT_REPLACEMENT), A, k)
    ev = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert not fb
    assert np.allclose(lam, ev[:k], rtol=1e-8)
    assert abs(metrics.trace_error(A, Uh, lam) - metrics.optimal_trace_error(A, k)) < 1e-9


def test_nystrom_exact_recovery_takes_fallback():
    """P9 + Remark 3.1: rank-k' SPD A makes Omega A Omega^T singular; fallback recovers A."""
    n, l, kk = 1024, 48, 20
    A = _spd(n, kk, 10, decay=lambda j: 1.0 / j)
    Uh, lam, fb = lowrank.nystrom(rng.Plan(n, 4, l, 11), A, kk)
    assert fb
    assert metrics.trace_error(A, Uh, lam) < 1e-10


def test_nystrom_identities():
    """P13: Z Z^T = Y (Omega Y)^{-1} Y^T, U_hat^T U_hat = I; step 6 as printed fails."""
    n, l, k = 1024, 64, 20
    A = _spd(n, 256, 12)
    # without replacement: rows of Omega are orthogonal (P3), so Omega A Omega^T
    # is non-singular; with replacement a repeated sample whose output signs
    # agree in every block gives two collinear rows and a singular matrix.
    plan = rng.Plan(n, 4, l, 13, rng.WITHOUT_REPLACEMENT)
    Y, Z, fb = lowrank.nystrom_factor(plan, A)
    assert not fb
    B = sketch.sketch(plan, Y)
    B = 0.5 * (B + B.T)
    assert metrics.rel_fro(Z @ Z.T, Y @ np.linalg.solve(B, Y.T)) < 1e-6
    Uh, lam, _ = lowrank.nystrom(plan, A, k)
    assert np.allclose(Uh.T @ Uh, np.eye(k), atol=1e-8)
    R = np.linalg.qr(Z, mode="r")
    _, St, VtT = np.linalg.svd(R)
    literal = Y @ (VtT.T[:, :k] / St[:k])
    assert np.max(np.abs(literal.T @ literal - np.eye(k))) > 1e-2


def test_collinear_rows_force_fallback():
    """With replacement, a repeated R_j whose Dt signs agree across all blocks makes
    two rows of Omega equal up to sign, so Omega A Omega^T is singular for any A."""
    n, p, l = 1024, 4, 64
    plan = rng.Plan(n, p, l, 13)
    Om = sketch.omega_explicit(plan)
    G = np.abs(Om @ Om.T) * l / n
    np.fill_diagonal(G, 0)
    pairs = np.argwhere(np.isclose(G, 1.0))
    assert len(pairs) > 0
    j, jj = pairs[0]
    assert plan.R[j] == plan.R[jj]
    A = _spd(n, 256, 12)
    _, _, fb = lowrank.nystrom_factor(plan, A)
    assert fb


def test_nystrom_near_optimal_and_bound():
    """P10/P11: trace error >= optimal and within eq. (3.10)'s bound with d = l/4."""
    n, l, k = 2048, 128, 40
    A = _spd(n, 512, 14)
    Uh, lam, fb = lowrank.nystrom(rng.Plan(n, 8, l, 15), A, k)
    err = metrics.trace_error(A, Uh, lam)
    opt = metrics.optimal_trace_error(A, k)
    tail_d = metrics.optimal_trace_error(A, l // 4)
    assert opt <= err * (1 + 1e-9) and err <= opt + 3 * tail_d
    assert err < 1.5 * opt


def test_shifted_nystrom_is_nystrom_of_the_shifted_matrix():
    """Shifting only the sketch, Y + nu Omega^T, is Algorithm 2 on A + nu I
    (formed explicitly here and run through the unshifted oracle) with nu
    subtracted from the eigenvalues."""
    n, p, l, k = 1024, 4, 64, 20
    A = _spd(n, 200, 3)
    plan = rng.Plan(n, p, l, 5)
    U, lam, nu, fb = lowrank.nystrom_shifted(plan, A, k, u=2.0 ** -24)
    assert nu > 0 and not fb
    U2, lam2, fb2 = lowrank.nystrom(plan, A + nu * np.eye(n), k, u=2.0 ** -24)
    assert np.allclose(lam, np.maximum(lam2 - nu, 0.0), rtol=1e-9, atol=1e-14)
    assert np.max(np.abs(U.T @ U - np.eye(k))) < 1e-10


def test_shifted_nystrom_needs_no_fallback_on_a_rank_deficient_matrix():
    """Rank 30 < l: Omega A Omega^T is singular (the unshifted method takes
    Remark 3.1's fallback); the shifted one factors it directly and still
    recovers A up to the shift's size.  (Sampling without replacement: with
    replacement two rows of Omega can be collinear, and then no shift of A
    makes Omega (A + nu I) Omega^T definite.)"""
    n, p, l, kk = 1024, 4, 48, 30
    A = _spd(n, kk, 7, decay=lambda j: 1.0 + 0.0 * j)
    plan = rng.Plan(n, p, l, 9, rng.WITHOUT_REPLACEMENT)
    _, _, fb0 = lowrank.nystrom(plan, A, kk)
    assert fb0
    U, lam, nu, fb = lowrank.nystrom_shifted(plan, A, kk)
    assert not fb
    assert np.linalg.norm(A - (U * lam) @ U.T) / np.linalg.norm(A) < 1e3 * nu
