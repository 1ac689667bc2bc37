"""Pins of the oracle's error measures (oracle/metrics.py) against values the
mathematics fixes, independently of the measures' own formulas.

* trace_error_structured (the trace-norm error of section 3.2 / Figure 1 for
  A = X diag(s) X^T + shift I, evaluated on span[X, U]) against the full
  eigendecomposition of the explicit n x n residual (metrics.trace_error) on
  small inputs, with and without a shift, with U inside and outside span X.
* ose_distortion (Definition 1.1's epsilon) on sketches whose singular values
  are known in closed form.
"""
import numpy as np
import pytest

from oracle import metrics


def _orth(n, d, rs):
    Q, _ = np.linalg.qr(rs.standard_normal((n, d)))
    return Q


@pytest.mark.parametrize("shift", [0.0, 1e-2])
@pytest.mark.parametrize("inside", [False, True])
def test_trace_error_structured_matches_explicit(shift, inside):
    rs = np.random.default_rng(5)
    n, d, k = 160, 24, 9
    X = _orth(n, d, rs)
    s = np.arange(1, d + 1, dtype=np.float64) ** -1.5
    A = (X * s) @ X.T + shift * np.eye(n)
    if inside:   # U spans part of range(X): an exact-recovery-like output
        U = X @ _orth(d, k, rs)
    else:
        U = _orth(n, k, rs)
    lam = np.sort(rs.uniform(0.05, 1.0, k))[::-1]
    want = metrics.trace_error(A, U, lam)
    got = metrics.trace_error_structured(X, s, U, lam, shift)
    assert abs(got - want) <= 1e-12 * max(1.0, want)


def test_trace_error_structured_optimum():
    """The top-k eigenpairs of X diag(s) X^T + shift I give the optimal trace
    error sum_{j>k}(s_j + shift) + shift (n - d), over sum(s) + n shift."""
    rs = np.random.default_rng(6)
    n, d, k, shift = 300, 40, 12, 3e-3
    X = _orth(n, d, rs)
    s = np.exp(-np.arange(d) / 8.0)
    got = metrics.trace_error_structured(X, s, X[:, :k], s[:k] + shift, shift)
    want = (np.sum(s[k:] + shift) + shift * (n - d)) / (np.sum(s) + n * shift)
    assert abs(got - want) <= 1e-12


def test_ose_distortion_closed_form():
    """Omega V with singular values (2, 1/2, 1): epsilon = max|sigma^2 - 1| = 3
    (a sigma in place of sigma^2 would give 1)."""
    rs = np.random.default_rng(7)
    n = 20
    Q = _orth(n, n, rs)
    V = _orth(n, 3, rs)
    # Omega = W diag(2, 1/2, 1, 1, ...) Q^T with Q's first columns = V's span
    Qv, _ = np.linalg.qr(np.concatenate([V, rs.standard_normal((n, n - 3))], axis=1))
    Qv[:, :3] = V
    W = _orth(n, n, rs)
    g = np.ones(n)
    g[:3] = [2.0, 0.5, 1.0]
    Omega = (W * g) @ Qv.T
    assert abs(metrics.ose_distortion(Omega, V) - 3.0) < 1e-12


def test_ose_distortion_scaled_isometry():
    """c Q for orthogonal Q: every sigma is c, epsilon = |c^2 - 1|."""
    rs = np.random.default_rng(8)
    n, d = 32, 5
    Q = _orth(n, n, rs)
    V = _orth(n, d, rs)
    for c in (0.5, 1.0, 1.3):
        assert abs(metrics.ose_distortion(c * Q, V) - abs(c * c - 1.0)) < 1e-12
