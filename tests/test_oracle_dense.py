"""Pins of the oracle's dense Gaussian / Rademacher sketches (the comparison
embeddings of section 4).

The Philox stream itself is pinned against numpy.random.Philox in
test_oracle_rng.py.  Here: the Box-Muller mapping is checked by inverting it
(radius and angle recover -2 ln u1 and 2 pi u2 from the output words), the
Gaussian entries pass distribution tests (moments, Kolmogorov-Smirnov, row
independence), Rademacher entries and column norms are exact, E[G^T G] = I,
and the subspace distortion of the generated G matches a numpy Gaussian's.
"""
import numpy as np
import pytest
import scipy.stats as st

from oracle import dense, metrics


def test_box_muller_inverts_to_the_words():
    words = dense.gaussian_words(11, 3, 64)             # 8 outputs x 4 words
    z = dense.box_muller(words).reshape(8, 4, 2)
    lo = (words & np.uint64(0xFFFFFFFF)).astype(np.float64)
    hi = (words >> np.uint64(32)).astype(np.float64)
    u1 = (lo + 0.5) / 2.0 ** 32
    u2 = (hi + 0.5) / 2.0 ** 32
    r2 = z[..., 0] ** 2 + z[..., 1] ** 2
    assert np.allclose(r2, -2.0 * np.log(u1), rtol=1e-13, atol=1e-13)
    ang = np.mod(np.arctan2(z[..., 1], z[..., 0]), 2.0 * np.pi)
    assert np.allclose(ang, 2.0 * np.pi * u2, rtol=0, atol=1e-12)


def test_gaussian_row_layout():
    """Entry x of a row comes from output x >> 3, word (x & 7) >> 1, cos for
    even x and sin for odd x."""
    n, l = 40, 9
    row = dense.gaussian_row(5, 2, n, l) * np.sqrt(l)
    words = dense.gaussian_words(5, 2, n)
    for x in [0, 1, 6, 7, 8, 17, 39]:
        w = int(words[x >> 3, (x & 7) >> 1])
        u1 = ((w & 0xFFFFFFFF) + 0.5) / 2.0 ** 32
        u2 = ((w >> 32) + 0.5) / 2.0 ** 32
        f = np.cos if x % 2 == 0 else np.sin
        assert abs(row[x] - np.sqrt(-2 * np.log(u1)) * f(2 * np.pi * u2)) < 1e-13


def test_gaussian_entries_are_standard_normal():
    G = dense.omega(dense.GAUSSIAN, 7, 16, 8192) * 4.0     # l = 16: undo 1/sqrt(l)
    x = G.ravel()
    N = x.size
    assert abs(x.mean()) < 5 / np.sqrt(N)
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0 / N)
    assert abs(st.kurtosis(x)) < 5 * np.sqrt(24.0 / N)
    assert st.kstest(x, "norm").pvalue > 1e-3
    C = np.corrcoef(G)
    off = C[~np.eye(16, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(8192)


def test_rademacher_entries_and_columns_exact():
    l, n = 24, 700
    G = dense.omega(dense.RADEMACHER, 3, l, n)
    assert np.all(np.abs(np.abs(G) - 1 / np.sqrt(l)) == 0)
    assert np.allclose(np.linalg.norm(G, axis=0), 1.0, rtol=0, atol=1e-15)
    assert 0.4 < np.mean(G > 0) < 0.6


@pytest.mark.parametrize("kind", [dense.GAUSSIAN, dense.RADEMACHER])
def test_expected_gram_is_identity(kind):
    """E[G^T G] = I over seeds (entries of variance 1/l, independent)."""
    n, l, T = 48, 16, 60
    acc = np.zeros((n, n))
    for seed in range(T):
        G = dense.omega(kind, seed, l, n)
        acc += G.T @ G
    acc /= T
    assert np.max(np.abs(np.diag(acc) - 1.0)) < 6 * np.sqrt(2.0 / (l * T))
    off = acc[~np.eye(n, dtype=bool)]
    assert np.max(np.abs(off)) < 6 / np.sqrt(l * T)


def test_gaussian_subspace_distortion_matches_numpy_gaussian():
    n, d, l = 1024, 10, 128
    rs = np.random.default_rng(4)
    V, _ = np.linalg.qr(rs.standard_normal((n, d)))
    ours = [metrics.ose_distortion(dense.omega(dense.GAUSSIAN, s, l, n), V) for s in range(8)]
    ref = [metrics.ose_distortion(rs.standard_normal((l, n)) / np.sqrt(l), V) for _ in range(8)]
    assert np.median(ours) < 1.3 * np.median(ref) and np.median(ours) > np.median(ref) / 1.3


def test_sketch_is_the_product():
    A = np.random.default_rng(1).standard_normal((100, 7))
    for kind in (dense.GAUSSIAN, dense.RADEMACHER):
        Y = dense.dense_sketch(kind, 9, 12, A)
        assert metrics.rel_fro(Y, dense.omega(kind, 9, 12, 100) @ A) < 1e-15


def test_pins_catch_a_swapped_half(monkeypatch):
    """Taking u1 from the high and u2 from the low half breaks the layout pin."""
    good = dense.box_muller

    def swapped(words):
        w = ((words & np.uint64(0xFFFFFFFF)) << np.uint64(32)) | (words >> np.uint64(32))
        return good(w)

    monkeypatch.setattr(dense, "box_muller", swapped)
    with pytest.raises(AssertionError):
        test_gaussian_row_layout()
