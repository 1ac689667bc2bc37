"""Pins of the oracle's single-view RSVD (section 3.3, Algorithm 3).

Pinned against an exact result (a rank-k' input is recovered to rounding and
its singular values come out exactly), against the special case of orthogonal
core sketches Phi and Psi, where the core solve reduces to C = Q^T A P and the
result to the truncated SVD of the projection Q Q^T A P P^T, formed here from
the closed-form Omega and Gamma, and against the optimal rank-k error.
Plausible mistakes planted in the bases or the core solve fail these pins.
"""
import numpy as np
import pytest

from oracle import rng, sketch, single_view as sv, metrics

WR, WOR = rng.WITH_REPLACEMENT, rng.WITHOUT_REPLACEMENT


def _plans(N1, N2, l, s, pl=(4, 4), ps=(4, 2), core_mode=WR, seed=10, range_mode=WR):
    """Omega (l x N2), Gamma (l x N1), Phi (s x N1), Psi (s x N2), independent seeds."""
    om = rng.Plan(N2, pl[0], l, seed, range_mode)
    ga = rng.Plan(N1, pl[1], l, seed + 1, range_mode)
    ph = rng.Plan(N1, ps[0], s, seed + 2, core_mode)
    ps_ = rng.Plan(N2, ps[1], s, seed + 3, core_mode)
    return om, ga, ph, ps_


def _lowrank(N1, N2, kk, seed):
    rs = np.random.default_rng(seed)
    return rs.standard_normal((N1, kk)) @ rs.standard_normal((kk, N2))


def _decaying(N1, N2, seed, decay=lambda j: j ** -2.0):
    rs = np.random.default_rng(seed)
    d = min(N1, N2)
    X, _ = np.linalg.qr(rs.standard_normal((N1, d)))
    W, _ = np.linalg.qr(rs.standard_normal((N2, d)))
    s = decay(np.arange(1, d + 1, dtype=np.float64))
    return (X * s) @ W.T


def _recon(U, S, V):
    return (U * S) @ V.T


def _exact_recovery_error(N1=256, N2=256, kk=30, l=40, s=80):
    A = _lowrank(N1, N2, kk, 3)
    U, S, V = sv.single_view(*_plans(N1, N2, l, s), A, kk)
    s_true = np.linalg.svd(A, compute_uv=False)[:kk]
    return metrics.rel_fro(_recon(U, S, V), A), float(np.max(np.abs(S - s_true)) / s_true[0])


def _orthogonal_core_error(N=256, l=48, k=20):
    """Phi, Psi orthogonal (p = 1, s = N, without replacement): the result must
    be the truncated SVD of Q Q^T A P P^T.  Omega and Gamma sample without
    replacement too, so that Y and X have full rank and the bases are unique
    up to rotation (with replacement two rows of a sketch can be collinear)."""
    A = _decaying(N, N, 5)
    om, ga, ph, ps_ = _plans(N, N, l, N, pl=(4, 4), ps=(1, 1), core_mode=WOR, range_mode=WOR)
    U, S, V = sv.single_view(om, ga, ph, ps_, A, k)
    Qr, _ = np.linalg.qr(A @ sketch.omega_explicit(om).T)
    Pr, _ = np.linalg.qr(A.T @ sketch.omega_explicit(ga).T)
    u, sg, vt = np.linalg.svd(Qr.T @ A @ Pr)
    ref = (Qr @ u[:, :k] * sg[:k]) @ (vt[:k] @ Pr.T)
    return metrics.rel_fro(_recon(U, S, V), ref), float(np.max(np.abs(S - sg[:k])) / sg[0])


@pytest.mark.parametrize("N1,N2", [(256, 256), (1024, 256), (256, 512)])
def test_exact_recovery(N1, N2):
    """A rank-k' input with k' <= l - 10 is recovered to rounding, with its
    exact singular values."""
    err, serr = _exact_recovery_error(N1, N2)
    assert err < 1e-10 and serr < 1e-12


def test_orthogonal_core_sketches_give_the_projected_truncated_svd():
    err, serr = _orthogonal_core_error()
    assert err < 1e-12 and serr < 1e-12


def test_error_close_to_optimal():
    """With l = 64 >= 3k and s = 2l the rank-20 error of a j^-2 spectrum stays
    within a small factor of the optimum (section 3.3 bounds it by the RSVD
    errors of A and A^T)."""
    N1, N2, l, s, k = 2048, 256, 64, 128, 20
    A = _decaying(N1, N2, 7)
    U, S, V = sv.single_view(*_plans(N1, N2, l, s, pl=(8, 4), ps=(8, 2)), A, k)
    opt = np.sqrt(np.sum(np.linalg.svd(A, compute_uv=False)[k:] ** 2)) / np.linalg.norm(A)
    err = metrics.rel_fro(_recon(U, S, V), A)
    assert opt <= err <= 1.5 * opt


def test_sketches_are_the_three_products():
    """Step 1 against the closed-form matrices."""
    N1, N2, l, s = 256, 128, 24, 40
    om, ga, ph, ps_ = _plans(N1, N2, l, s, pl=(2, 4), ps=(4, 2))
    A = np.random.default_rng(2).standard_normal((N1, N2))
    X, Y, Z = sv.sketches(om, ga, ph, ps_, A)
    E = sketch.omega_explicit
    assert metrics.rel_fro(X, A.T @ E(ga).T) < 1e-13
    assert metrics.rel_fro(Y, A @ E(om).T) < 1e-13
    assert metrics.rel_fro(Z, E(ph) @ A @ E(ps_).T) < 1e-13


def test_rank_deficient_sketch_keeps_only_its_range():
    """p = 1 with replacement and l close to r repeats samples: Y has collinear
    columns, and Q spans exactly range(Y) (its projector fixes Y)."""
    N1, N2, l, s = 512, 64, 48, 64
    om, ga, ph, ps_ = _plans(N1, N2, l, s, pl=(1, 1), ps=(1, 1))
    assert len(set(om.R.tolist())) < l
    A = _decaying(N1, N2, 9)
    X, Y, Z = sv.sketches(om, ga, ph, ps_, A)
    Q, P = sv.bases(X, Y)
    assert Q.shape[1] == np.linalg.matrix_rank(Y) < l
    assert metrics.rel_fro(Q @ (Q.T @ Y), Y) < 1e-13
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-13


MUTATIONS = {
    "bases_swapped": lambda X, Y: tuple(np.linalg.qr(M, mode="reduced")[0] for M in (X, Y)),
    "core_transpose_for_pinv": lambda PhQ, Z, PsP: PhQ.T @ Z @ PsP,
    "core_right_pinv_missing": lambda PhQ, Z, PsP: np.linalg.lstsq(PhQ, Z, rcond=None)[0] @ PsP,
    "core_sides_swapped": lambda PhQ, Z, PsP: np.linalg.lstsq(
        PhQ, np.linalg.lstsq(PsP, Z.T, rcond=None)[0].T, rcond=None)[0].T,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistakes(name, monkeypatch):
    target = "bases" if name.startswith("bases") else "core_matrix"
    monkeypatch.setattr(sv, target, MUTATIONS[name])
    e1, s1 = _exact_recovery_error()
    e2, s2 = _orthogonal_core_error()
    assert max(e1, s1) > 1e-6 or max(e2, s2) > 1e-6
