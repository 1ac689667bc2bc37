"""Pins of the oracle's block SRHT (section 2, eq. (2.1)-(2.4)).

Each test checks the oracle against something other than itself: a library
routine (scipy.linalg.hadamard, numpy.kron), a closed form, an invariant the
paper's definition fixes, a special case that reduces to a textbook object,
or a Monte Carlo expectation.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import rng, sketch, metrics


@pytest.mark.parametrize("r", [1, 2, 4, 32, 256])
def test_fwht_is_sylvester_hadamard(r):
    """P1: FWHT(e_k) is column k of the Sylvester matrix (scipy's, and kron)."""
    H = sketch.fwht_rows(np.eye(r))
    assert np.array_equal(H, sla.hadamard(r).astype(np.float64))
    K = np.ones((1, 1))
    while K.shape[0] < r:
        K = np.kron(K, np.array([[1.0, 1.0], [1.0, -1.0]]))
    assert np.array_equal(H, K)


def test_fwht_involution_and_kronecker():
    """P1: H_r H_r = r I and H_a (x) H_b = H_ab for the x = x_hi*b + x_lo split."""
    rs = np.random.default_rng(0)
    X = rs.standard_normal((64, 5))
    assert np.allclose(sketch.fwht_rows(sketch.fwht_rows(X)), 64 * X, atol=1e-12)
    Ha, Hb = sla.hadamard(8), sla.hadamard(16)
    assert np.array_equal(np.kron(Ha, Hb), sla.hadamard(128))
    y = np.arange(128)[:, None]
    x = np.arange(128)[None, :]
    assert np.array_equal(sketch.hadamard_sign(y, x), sla.hadamard(128))


CASES = [
    (64, 1, 16, rng.WITH_REPLACEMENT),
    (64, 4, 16, rng.WITH_REPLACEMENT),
    (256, 8, 48, rng.WITH_REPLACEMENT),
    (256, 2, 100, rng.WITHOUT_REPLACEMENT),
    (512, 512, 20, rng.WITH_REPLACEMENT),   # r = 1
    (128, 4, 128, rng.WITH_REPLACEMENT),    # l > r
]


@pytest.mark.parametrize("n,p,l,mode", CASES)
def test_explicit_equals_fwht(n, p, l, mode):
    """Closed-form Omega @ A equals per-block FWHT + sample + signs + sum."""
    plan = rng.Plan(n, p, l, 3, mode)
    A = np.random.default_rng(1).standard_normal((n, 7))
    Y1 = sketch.omega_explicit(plan) @ A
    Y2 = sketch.sketch(plan, A)
    assert metrics.rel_fro(Y2, Y1) < 1e-13


@pytest.mark.parametrize("n,p,l,mode", CASES)
def test_entries_and_column_norms(n, p, l, mode):
    """P2: every entry is +-1/sqrt(l) and every column has norm exactly 1."""
    Om = sketch.omega_explicit(rng.Plan(n, p, l, 4, mode))
    assert np.allclose(np.abs(Om), 1.0 / np.sqrt(l), rtol=0, atol=1e-15)
    assert np.allclose(np.linalg.norm(Om, axis=0), 1.0, atol=1e-14)


@pytest.mark.parametrize("n,p,l,mode", CASES)
def test_gram_of_rows_closed_form(n, p, l, mode):
    """P3: (Omega Omega^T)_{jj'} = (r/l) [R_j = R_j'] sum_i Dt_j Dt_j'."""
    plan = rng.Plan(n, p, l, 5, mode)
    Om = sketch.omega_explicit(plan)
    G = Om @ Om.T
    same = (plan.R[:, None] == plan.R[None, :]).astype(np.float64)
    expect = (plan.r / l) * same * (plan.Dt.T @ plan.Dt)
    assert np.allclose(G, expect, atol=1e-12)
    assert np.allclose(np.diag(G), n / l, atol=1e-12)
    if mode == rng.WITHOUT_REPLACEMENT:
        assert np.allclose(G, (n / l) * np.eye(l), atol=1e-12)


@pytest.mark.parametrize("n", [8, 64, 1024])
def test_srht_permutation_is_orthogonal(n):
    """P4: p = 1, l = r = n without replacement: Omega is orthogonal."""
    plan = rng.Plan(n, 1, n, 6, rng.WITHOUT_REPLACEMENT)
    Om = sketch.omega_explicit(plan)
    assert np.allclose(Om.T @ Om, np.eye(n), atol=1e-12)
    x = np.random.default_rng(2).standard_normal(n)
    assert abs(np.linalg.norm(sketch.sketch(plan, x[:, None])) - np.linalg.norm(x)) < 1e-12


def test_r_equals_one_is_rademacher():
    """P5: r = 1 reduces to a Rademacher matrix with entries Dt^(i)_j D^(i)_0 / sqrt(l)."""
    n, l = 64, 10
    plan = rng.Plan(n, n, l, 8)
    Om = sketch.omega_explicit(plan)
    expect = (plan.Dt * plan.D[:, 0][:, None]).T / np.sqrt(l)
    assert np.array_equal(Om, expect)


def test_block_linearity_and_subsample():
    """P6: eq. (2.4) sum of block contributions; p = 1 plan on A^(1) is block 1."""
    n, p, l, r = 1024, 4, 64, 256
    plan = rng.Plan(n, p, l, 9)
    A = np.random.default_rng(3).standard_normal((n, 5))
    parts = []
    for i in range(p):
        Ai = np.zeros_like(A)
        Ai[i * r:(i + 1) * r] = A[i * r:(i + 1) * r]
        parts.append(sketch.sketch(plan, Ai))
    assert metrics.rel_fro(sum(parts), sketch.sketch(plan, A)) < 1e-14
    sub = rng.Plan(r, 1, l, 9)
    assert metrics.rel_fro(sketch.sketch(sub, A[:r]), parts[0]) < 1e-14


def test_expected_gram_is_identity():
    """P7: E[Omega^T Omega] = I; diagonal exactly 1 per draw, off-diagonal mean ~ 0."""
    n, p, l, T = 64, 4, 8, 400
    acc = np.zeros((n, n))
    for s in range(T):
        Om = sketch.omega_explicit(rng.Plan(n, p, l, 1000 + s))
        G = Om.T @ Om
        assert np.allclose(np.diag(G), 1.0, atol=1e-14)
        acc += G
    acc /= T
    off = acc - np.diag(np.diag(acc))
    assert np.max(np.abs(off)) < 6.0 / np.sqrt(l * T)


def test_ose_distortion_like_gaussian():
    """P8 (Def. 1.1): distortion on random d-dim subspaces is close to a Gaussian's."""
    n, p, l, d = 1024, 8, 128, 10
    rs = np.random.default_rng(4)
    eb, eg = [], []
    for t in range(30):
        V, _ = np.linalg.qr(rs.standard_normal((n, d)))
        Om = sketch.omega_explicit(rng.Plan(n, p, l, 500 + t))
        G = rs.standard_normal((l, n)) / np.sqrt(l)
        eb.append(metrics.ose_distortion(Om, V))
        eg.append(metrics.ose_distortion(G, V))
    mb, mg = np.median(eb), np.median(eg)
    assert mb < 1.5 * mg and mb < 1.0


def test_sketch_entry_matches_sketch():
    plan = rng.Plan(2048, 4, 40, 12)
    A = np.random.default_rng(5).standard_normal((2048, 3))
    Y = sketch.sketch(plan, A)
    for j, c in [(0, 0), (7, 1), (39, 2), (20, 0)]:
        assert abs(sketch.sketch_entry(plan, A[:, c], j) - Y[j, c]) < 1e-12 * np.abs(Y).max()


@pytest.mark.parametrize("n,p,l,m,chunk", [(4096, 8, 64, 37, 8), (2048, 1, 40, 5, 256),
                                           (3000, 6, 24, 19, 4)])
def test_sketch_parallel_is_bitwise_sketch(n, p, l, m, chunk):
    """The block-parallel evaluation (threads over blocks and column slices)
    gives bitwise the sequential oracle sketch (same terms, same block order)."""
    plan = rng.Plan(n, p, l, 3)
    A = np.random.default_rng(6).standard_normal((n, m)).astype(np.float32)
    assert np.array_equal(sketch.sketch_parallel(plan, A, workers=4, col_chunk=chunk),
                          sketch.sketch(plan, A))


PADDED_CASES = [
    # n, p, l, mode  -- block sizes r that are not powers of two (partial SRHT)
    (300, 3, 20, rng.WITH_REPLACEMENT),      # r = 100 -> 128
    (1000, 8, 40, rng.WITH_REPLACEMENT),     # r = 125 -> 128
    (96, 1, 30, rng.WITHOUT_REPLACEMENT),    # r = 96 -> 128, l <= r'
    (770, 5, 64, rng.WITH_REPLACEMENT),      # r = 154 -> 256
    (7, 7, 5, rng.WITH_REPLACEMENT),         # r = 1 (no padding)
    (513, 1, 9, rng.WITH_REPLACEMENT),       # r = 513 -> 1024
]


def _pad_blocks(A, p, r, rp):
    """A with rp - r zero rows appended to each of its p blocks of r rows."""
    out = np.zeros((p * rp,) + A.shape[1:])
    for i in range(p):
        out[i * rp:i * rp + r] = A[i * r:(i + 1) * r]
    return out


@pytest.mark.parametrize("n,p,l,mode", PADDED_CASES)
def test_partial_srht_explicit_equals_padded_fwht(n, p, l, mode):
    """Section 2's partial SRHT: the closed form restricted to the r real
    columns of each block equals the FWHT path on zero-padded blocks, and every
    entry is +-1/sqrt(l) with unit columns."""
    plan = rng.Plan(n, p, l, 5, mode)
    Om = sketch.omega_explicit(plan)
    A = np.random.default_rng(3).standard_normal((n, 6))
    assert metrics.rel_fro(sketch.sketch(plan, A), Om @ A) < 1e-13
    assert np.all(np.abs(np.abs(Om) * np.sqrt(l) - 1.0) < 1e-15)
    assert np.allclose(np.linalg.norm(Om, axis=0), 1.0, atol=1e-14)


@pytest.mark.parametrize("n,p,l,mode", PADDED_CASES)
def test_partial_srht_is_the_power_of_two_plan_on_padded_input(n, p, l, mode):
    """The tables are keyed by (block, index): a plan with r rows per block is
    the (p r', p) plan on the input with zero rows appended to every block."""
    plan = rng.Plan(n, p, l, 11, mode)
    r, rp = plan.r, plan.rp
    full = rng.Plan(p * rp, p, l, 11, mode)
    assert np.array_equal(plan.R, full.R)
    assert np.array_equal(plan.D_bits, full.D_bits[:, :r])
    A = np.random.default_rng(4).standard_normal((n, 5))
    assert metrics.rel_fro(sketch.sketch(plan, A), sketch.sketch(full, _pad_blocks(A, p, r, rp))) < 1e-14


def test_partial_srht_pin_catches_padding_at_the_end(monkeypatch):
    """Padding the whole input at its end instead of each block fails the
    explicit-form pin."""
    plan = rng.Plan(300, 3, 20, 5)

    def bad_partial(pl, AA, i):
        Apad = np.zeros((pl.p * pl.rp,) + AA.shape[1:])
        Apad[:pl.n] = AA
        Ai = Apad[i * pl.rp:(i + 1) * pl.rp]
        B = sketch.fwht_rows(np.concatenate([pl.D[i], np.ones(pl.rp - pl.r)])[:, None] * Ai)
        return pl.Dt[i][:, None] * B[pl.R, :]

    A = np.random.default_rng(3).standard_normal((300, 4))
    ref = sketch.omega_explicit(plan) @ A
    monkeypatch.setattr(sketch, "block_partial", bad_partial)
    assert metrics.rel_fro(sketch.sketch(plan, A), ref) > 1e-3


@pytest.mark.parametrize("n,p,l,mode", CASES)
def test_right_sketch_is_omega_applied_from_the_right(n, p, l, mode):
    """A Omega^T (Algorithm 1's orientation) equals the closed-form Omega
    multiplied from the right, entry by entry; the rows are independent."""
    plan = rng.Plan(n, p, l, 8, mode)
    A = np.random.default_rng(2).standard_normal((5, n))
    Y = sketch.sketch_right(plan, A)
    assert Y.shape == (5, l)
    assert metrics.rel_fro(Y, A @ sketch.omega_explicit(plan).T) < 1e-13
    assert metrics.rel_fro(sketch.sketch_right(plan, A[3:4]), Y[3:4]) < 1e-15


def test_right_sketch_entry_matches():
    plan = rng.Plan(2048, 4, 40, 12)
    A = np.random.default_rng(7).standard_normal((3, 2048))
    Y = sketch.sketch_right(plan, A)
    for g, j in [(0, 0), (1, 7), (2, 39), (0, 20)]:
        assert abs(sketch.sketch_right_entry(plan, A[g], j) - Y[g, j]) < 1e-12 * np.abs(Y).max()


@pytest.mark.parametrize("mutation", ["drop_D", "drop_Dt", "swap_blocks", "no_scale",
                                      "skip_stage", "lo_hi_swap"])
def test_pins_catch_planted_mistakes(mutation, monkeypatch):
    """A plausible mistake planted in the oracle's FWHT path fails a pin."""
    plan = rng.Plan(256, 4, 32, 13)
    A = np.random.default_rng(6).standard_normal((256, 4))
    ref = sketch.omega_explicit(plan) @ A
    good_fwht = sketch.fwht_rows

    def bad_partial(pl, AA, i):
        r = pl.r
        Ai = np.asarray(AA[i * r:(i + 1) * r], dtype=np.float64)
        D = pl.D[i] if mutation != "drop_D" else np.ones(r)
        Dt = pl.Dt[i] if mutation != "drop_Dt" else np.ones(pl.l)
        if mutation == "swap_blocks":
            Ai = np.asarray(AA[(pl.p - 1 - i) * r:(pl.p - i) * r], dtype=np.float64)
        B = D[:, None] * Ai
        if mutation == "skip_stage":
            h = 1
            while h < r // 2:          # the last butterfly stage is left out
                V = B.reshape(r // (2 * h), 2, h, -1)
                u, v = V[:, 0].copy(), V[:, 1].copy()
                V[:, 0], V[:, 1] = u + v, u - v
                h *= 2
        elif mutation == "lo_hi_swap":
            B = good_fwht(B)[np.argsort(np.arange(r)[::-1])]
        else:
            B = good_fwht(B)
        out = Dt[:, None] * B[pl.R, :]
        return out * (np.sqrt(pl.l) if mutation == "no_scale" else 1.0)

    monkeypatch.setattr(sketch, "block_partial", bad_partial)
    assert metrics.rel_fro(sketch.sketch(plan, A), ref) > 1e-3
