"""GPU parity of the randomized SVD (Algorithm 1) and Nystrom (Algorithm 2)
against the FP64 oracle run with the same Omega (same plan and seed).

Pass rule: the GPU's approximation error is within 1% of the oracle's
(err_gpu <= 1.01 err_oracle); singular vectors are compared through
reconstructions and orthonormality, not entry by entry (they are unique only
up to sign and rotation within repeated values)."""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, lowrank, metrics
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu


def _rsvd_case(n, m, p, l, k, A, seed, mode=0, precision=bs.FP32):
    dev = device()
    plan = bs.Plan(n, p, l, seed, mode, precision=precision, device=dev)
    U, S, V, info = bs.rsvd(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.lowrank_fro_error(Ah, to64(U), to64(S), to64(V))
    Uo, So, Vo = lowrank.rsvd(rng.Plan(n, p, l, seed, mode), Ah, k)
    err_o = metrics.lowrank_fro_error(Ah, Uo, So, Vo)
    return U, S, V, int(info.item()), err, err_o, So


@pytest.mark.parametrize("n,m,p,l,k", [
    (4096, 256, 4, 128, 50),    # the small RSVD workload
    (8192, 100, 8, 64, 20),     # ragged m
    (4096, 300, 16, 37, 11),    # odd l
    (2048, 64, 4, 128, 16),     # l >= m: Q = I
    (20000, 300, 16, 100, 30),  # Gram of Z on the int8 digit path: ragged rows and columns
])
def test_rsvd_matches_oracle(n, m, p, l, k):
    dev = device()
    say("rsvd", n, m, p, l, k)
    A = workloads.lowrank_tall(n, m, "inv_sq", 3, device=dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 7)
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert err <= 1.01 * err_o
    assert np.allclose(to64(S), So, rtol=2e-4, atol=1e-6 * So[0])
    Uh, Vh = to64(U), to64(V)
    assert np.max(np.abs(Uh.T @ Uh - np.eye(k))) < 1e-4
    assert np.max(np.abs(Vh.T @ Vh - np.eye(k))) < 1e-4
    assert info == 0
    Sh = to64(S)
    assert np.all(np.diff(Sh) <= 0)


@pytest.mark.parametrize("n,m,p,l,k", [
    (8192, 1500, 2, 1100, 50),    # SVD of R on 1120 columns: streamed 32-column pairs
    (8192, 2600, 1, 2200, 40),    # 2208 columns: streamed 32-column pairs
    (4096, 900, 4, 700, 30),      # 704 columns: 16-column pairs staged in LDS
    (16400, 900, 4, 700, 30),     # and the int8 Gram of Z over 700 columns (66 tiles)
])
def test_rsvd_large_sketch_sizes(n, m, p, l, k):
    """Sketch sizes that take both forms of the Jacobi SVD's block step."""
    dev = device()
    say("rsvd large l", n, m, p, l, k)
    A = workloads.gaussian_cols(n, m, "pow1.5", n + m + l, device=dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 17)
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert info & bs.INFO_JACOBI_NOCONV == 0
    assert err <= 1.01 * err_o


def test_rsvd_full_range_is_truncated_svd():
    dev = device()
    n, m, p, l, k = 2048, 64, 4, 128, 16
    A = workloads.lowrank_tall(n, m, "inv_sq", 4, device=dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 8)
    opt = metrics.optimal_fro_error(to64(A), k)
    assert abs(err - opt) < 1e-5 * max(opt, 1e-3)


def test_rsvd_exact_recovery():
    """P9: rank-30 input with l = 64 is recovered to FP32 accuracy."""
    dev = device()
    n, m, p, l, k = 4096, 128, 4, 64, 30
    g = torch.Generator(device="cpu").manual_seed(5)
    X = torch.randn(n, 30, generator=g, dtype=torch.float64)
    W = torch.randn(m, 30, generator=g, dtype=torch.float64)
    A = (X @ W.T).to(torch.float32).to(dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 9)
    say("  exact recovery err", err, "info", info)
    assert err < 1e-5


def test_rsvd_rank_clamped():
    """k above min(l, m): the tail of S, U and the flag report the clamp."""
    dev = device()
    n, m, p, l, k = 2048, 48, 4, 32, 40
    A = workloads.lowrank_tall(n, m, "inv_sq", 6, device=dev)
    plan = bs.Plan(n, p, l, 10, device=dev)
    U, S, V, info = bs.rsvd(plan, A, k)
    torch.cuda.synchronize()
    Sh = to64(S)
    assert int(info.item()) & bs.INFO_RANK_CLAMPED
    assert np.all(Sh[32:] == 0) and np.all(Sh[:32] > 0)
    assert torch.all(U[:, 32:] == 0)


def test_rsvd_subsample_of_large_workload():
    """The first 2^16 rows of the 2^20 x 1024 workload as a p = 1 plan
    (l = 512, rank 256): GPU error within 1% of the FP64 oracle's."""
    dev = device()
    cfg = workloads.CONFIGS["c2_fp32_apply"]
    r = cfg["n"] // cfg["p"]
    A = workloads.lowrank_tall(cfg["n"], cfg["m"], cfg["spectrum"], cfg["seed"], device=dev)
    Asub = A[:r].contiguous()
    del A
    say("subsample rsvd", r, cfg["m"], cfg["l"], cfg["k"])
    U, S, V, info, err, err_o, So = _rsvd_case(r, cfg["m"], 1, cfg["l"], cfg["k"], Asub,
                                               cfg["seed"])
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert err <= 1.01 * err_o


def test_rsvd_split_bf16_subsample():
    """Rank-256 RSVD (l = 512) of A_sub = A[0:2^16] of the split-BF16 sketch
    workload with the sketch on BF16 matrix cores: within 1% of the FP64
    oracle's error."""
    dev = device()
    cfg = workloads.CONFIGS["c3_split_bf16"]
    r = cfg["n"] // cfg["p"]
    A = workloads.lowrank_tall(cfg["n"], cfg["m"], cfg["spectrum"], cfg["seed"], device=dev)
    Asub = A[:r].contiguous()
    del A
    say("subsample rsvd split-bf16", r, cfg["m"], cfg["l"], cfg["k"])
    U, S, V, info, err, err_o, So = _rsvd_case(r, cfg["m"], 1, cfg["l"], cfg["k"], Asub,
                                               cfg["seed"], precision=bs.SPLIT_BF16)
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert err <= 1.01 * err_o


@pytest.mark.parametrize("lda_pad", [1, 4, 30])
def test_rsvd_product_forms_agree(lda_pad):
    """The tall products Z = A Q and U = Z M run on split-BF16 matrix cores
    with six products when A's rows are 16-byte aligned (lda a multiple of 4)
    and on the FP32 matrix cores otherwise.  The same A, once contiguous
    (m = 100, aligned) and once as a view with lda = 100 + lda_pad (101 and
    130: the FP32 form; 104: the split form with a strided A): both within 1%
    of the oracle, and their rank-k approximations equal to FP32 accuracy."""
    dev = device()
    n, m, p, l, k = 8192, 100, 8, 64, 20
    say("rsvd product forms", n, m, p, l, k, "lda", m + lda_pad)
    A = workloads.lowrank_tall(n, m, "inv_sq", 13, device=dev)
    big = torch.zeros(n, m + lda_pad, device=dev)
    big[:, :m] = A
    Av = big[:, :m]
    assert Av.stride(0) == m + lda_pad
    plan = bs.Plan(n, p, l, 19, device=dev)
    Ua, Sa, Va, _ = bs.rsvd(plan, A, k)
    Ub, Sb, Vb, _ = bs.rsvd(plan, Av, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    Uo, So, Vo = lowrank.rsvd(rng.Plan(n, p, l, 19), Ah, k)
    err_o = metrics.lowrank_fro_error(Ah, Uo, So, Vo)
    for U, S, V in ((Ua, Sa, Va), (Ub, Sb, Vb)):
        assert metrics.lowrank_fro_error(Ah, to64(U), to64(S), to64(V)) <= 1.01 * err_o
    Ra = (to64(Ua) * to64(Sa)) @ to64(Va).T
    Rb = (to64(Ub) * to64(Sb)) @ to64(Vb).T
    assert metrics.rel_fro(Ra, Rb) < 1e-5


@pytest.mark.parametrize("n,m,p,l,k,precision", [
    (96, 20, 1, 16, 5, bs.FP32),          # fewer rows than one 128-row tile, K = 20 < 32
    (256, 12, 2, 8, 1, bs.FP32),          # rank 1, K = 12 (one partial quad row)
    (1000, 36, 8, 24, 24, bs.FP32),       # ragged rows (1000 = 7 * 128 + 104), k = l
    (640, 44, 4, 40, 7, bs.SPLIT_BF16),   # three products on a ragged shape
])
def test_rsvd_small_shapes(n, m, p, l, k, precision):
    """Shapes at the edges of the tall-product kernel's tiles (rows, k tail,
    columns): within 1% of the oracle's error.  The samples are drawn without
    replacement: with l of ~128 rows drawn with replacement a repeated row is
    likely, and the sketch's range then has fewer than l directions (the GPU
    keeps the range's directions, the oracle's QR adds an arbitrary one)."""
    dev = device()
    say("rsvd small", n, m, p, l, k, precision)
    A = workloads.lowrank_tall(n, m, "inv_sq", 5, device=dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 23, mode=rng.WITHOUT_REPLACEMENT,
                                               precision=precision)
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert err <= 1.01 * err_o


@pytest.mark.parametrize("n,m,p,l,k", [
    (4096, 300, 16, 37, 11),    # ragged k tail of both products
    (8192, 100, 8, 64, 20),
])
def test_rsvd_split_bf16_matches_oracle(n, m, p, l, k):
    """Split-BF16 plans: sketch and tall products (three products) on BF16
    matrix cores, error within 1% of the FP64 oracle's."""
    dev = device()
    say("rsvd split-bf16", n, m, p, l, k)
    A = workloads.lowrank_tall(n, m, "inv_sq", 3, device=dev)
    U, S, V, info, err, err_o, So = _rsvd_case(n, m, p, l, k, A, 7, precision=bs.SPLIT_BF16)
    say("  err gpu", err, "oracle", err_o, "info", info)
    assert err <= 1.01 * err_o
    Uh = to64(U)
    assert np.max(np.abs(Uh.T @ Uh - np.eye(k))) < 1e-3


def test_nystrom_split_bf16():
    dev = device()
    n, p, l, k = 4096, 4, 256, 64
    say("nystrom split-bf16", n, p, l, k)
    A = workloads.spd(n, 512, "inv_sq", 11, device=dev)
    U, lam, info, err, err_o, lo, fb = _nys_case(n, p, l, k, A, 12, rng.WITHOUT_REPLACEMENT,
                                                 precision=bs.SPLIT_BF16)
    say("  err gpu", err, "oracle", err_o, "info", info, "oracle fallback", fb)
    assert err <= 1.01 * err_o


def _nys_case(n, p, l, k, A, seed, mode=0, precision=bs.FP32):
    dev = device()
    plan = bs.Plan(n, p, l, seed, mode, precision=precision, device=dev)
    U, lam, info = bs.nystrom(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.trace_error(Ah, to64(U), to64(lam))
    Uo, lo, fb = lowrank.nystrom(rng.Plan(n, p, l, seed, mode), Ah, k)
    err_o = metrics.trace_error(Ah, Uo, lo)
    return U, lam, int(info.item()), err, err_o, lo, fb


@pytest.mark.parametrize("n,p,l,k,spec", [
    (4096, 4, 256, 64, "inv_sq"),
    (2048, 8, 128, 40, "inv_sq"),
    (4096, 16, 200, 50, "pow1.5"),
])
def test_nystrom_matches_oracle(n, p, l, k, spec):
    dev = device()
    say("nystrom", n, p, l, k, spec)
    A = workloads.spd(n, 512, spec, 11, device=dev)
    U, lam, info, err, err_o, lo, fb = _nys_case(n, p, l, k, A, 12, rng.WITHOUT_REPLACEMENT)
    say("  err gpu", err, "oracle", err_o, "info", info, "oracle fallback", fb)
    assert err <= 1.01 * err_o
    Uh = to64(U)
    assert np.max(np.abs(Uh.T @ Uh - np.eye(k))) < 1e-3
    assert np.allclose(to64(lam), lo, rtol=1e-3)


def test_nystrom_orthogonal_omega():
    """p = 1, l = r = n without replacement: Nystrom gives the top eigenpairs."""
    dev = device()
    n, k = 512, 16
    A = workloads.spd(n, n, "inv_sq", 13, device=dev)
    U, lam, info, err, err_o, lo, fb = _nys_case(n, 1, n, k, A, 14, rng.WITHOUT_REPLACEMENT)
    ev = np.sort(np.linalg.eigvalsh(to64(A)))[::-1]
    assert np.allclose(to64(lam), ev[:k], rtol=1e-4)
    assert err <= 1.01 * err_o


def test_nystrom_fallback_exact_recovery():
    """Rank-20 SPD input with l = 48: Omega A Omega^T is singular, the
    Remark 3.1 fallback is taken and A is recovered to FP32 accuracy."""
    dev = device()
    n, p, l, k = 2048, 4, 48, 20
    A = workloads.spd(n, 20, "inv_sq", 15, device=dev)
    U, lam, info, err, err_o, lo, fb = _nys_case(n, p, l, k, A, 16)
    say("  fallback err", err, "info", info)
    assert info & bs.INFO_CHOL_FALLBACK
    assert err < 1e-4


@pytest.mark.parametrize("n,p,l,k,spec", [
    (4096, 4, 256, 64, "inv_sq"),
    (2048, 8, 128, 40, "inv_sq"),
    (4096, 16, 200, 50, "pow1.5"),
])
def test_nystrom_shifted_matches_oracle(n, p, l, k, spec):
    """Shifted Nystrom (A + nu I, nu = sqrt(n) 2^-24 ||Y||_F for the FP32
    sketch) against the oracle's shifted Nystrom with the same rule."""
    dev = device()
    say("nystrom shifted", n, p, l, k, spec)
    A = workloads.spd(n, 512, spec, 11, device=dev)
    plan = bs.Plan(n, p, l, 12, rng.WITHOUT_REPLACEMENT, device=dev)
    U, lam, info = bs.nystrom_shifted(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.trace_error(Ah, to64(U), to64(lam))
    Uo, lo, nu, fb = lowrank.nystrom_shifted(rng.Plan(n, p, l, 12, rng.WITHOUT_REPLACEMENT), Ah, k,
                                             u=2.0 ** -24)
    err_o = metrics.trace_error(Ah, Uo, lo)
    say("  err gpu", err, "oracle", err_o, "nu", nu, "info", int(info.item()))
    assert err <= 1.01 * err_o
    assert not fb and int(info.item()) == 0
    assert np.allclose(to64(lam), lo, rtol=1e-3, atol=1e-3 * lo[0])
    Uh = to64(U)
    assert np.max(np.abs(Uh.T @ Uh - np.eye(k))) < 1e-3


def test_nystrom_shifted_needs_no_fallback():
    """Rank-20 SPD input with l = 48 (sampled without replacement): the
    unshifted method needs Remark 3.1's fallback, the shifted one factors
    directly.  Its error is the shift's (nu ~ 2.5e-6 here, at FP32 sketch
    precision, against eigenvalues down to 1/400): both sides give ~2e-3, and
    the GPU must stay within 1% of the oracle's shifted result."""
    dev = device()
    n, p, l, k = 2048, 4, 48, 20
    A = workloads.spd(n, 20, "inv_sq", 15, device=dev)
    plan = bs.Plan(n, p, l, 16, rng.WITHOUT_REPLACEMENT, device=dev)
    U, lam, info = bs.nystrom_shifted(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.trace_error(Ah, to64(U), to64(lam))
    Uo, lo, nu, fb = lowrank.nystrom_shifted(rng.Plan(n, p, l, 16, rng.WITHOUT_REPLACEMENT), Ah,
                                             k, u=2.0 ** -24)
    err_o = metrics.trace_error(Ah, Uo, lo)
    say("  shifted rank-20 err", err, "oracle", err_o, "info", int(info.item()))
    assert int(info.item()) & bs.INFO_CHOL_FALLBACK == 0 and not fb
    assert err <= 1.01 * err_o
