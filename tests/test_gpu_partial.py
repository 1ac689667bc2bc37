"""GPU parity of the partial block SRHT (block sizes r that are not powers of
two; section 2: the first r columns of an SRHT of size r' = the next power of
two, i.e. each block padded with zeros) against the FP64 oracle.

Tables bit-exact (D in the padded layout: bit i*r' + x); the FP32 sketch
within 1e-5; the padded identity against the power-of-two plan on a padded
copy of A; the right-side sketch, the randomized SVD and the Nystrom
approximation on such plans."""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch, lowrank, metrics
from tests.gpu_util import device, to64, unpack_bits, say

pytestmark = pytest.mark.gpu

TOL = 1e-5

PARTIAL_CASES = [
    # n, p, l, m, mode      r -> r': what it exercises
    (300, 3, 20, 70, 0),     # 100 -> 128: one 128-row chunk per block, partial waves
    (1000, 8, 40, 65, 0),    # 125 -> 128
    (770, 5, 64, 33, 0),     # 154 -> 256: chunk 256
    (4000, 4, 96, 130, 0),   # 1000 -> 1024: chunk 512, second chunk partial
    (12000, 4, 600, 40, 0),  # 3000 -> 4096: 16-wave kernel, 6 chunks per block
    (150, 3, 16, 9, 0),      # 50 -> 64: chunk 64, waves 6 and 7 past the rows
    (60, 3, 7, 20, 0),       # 20 -> 32: direct kernel
    (300, 3, 120, 17, 1),    # without replacement, l > r (l <= r')
]


@pytest.mark.parametrize("n,p,l,m,mode", PARTIAL_CASES)
def test_partial_tables_and_sketch(n, p, l, m, mode):
    dev = device()
    say("partial", n, p, l, m, mode)
    seed = 300 + n + l
    plan = bs.Plan(n, p, l, seed, mode, device=dev)
    op = rng.Plan(n, p, l, seed, mode)
    R, Db, Dtb = plan.export()
    assert np.array_equal(R.astype(np.int64), op.R)
    bits = unpack_bits(Db, p * op.rp).reshape(p, op.rp)[:, :op.r]
    assert np.array_equal(bits, op.D_bits)
    A = workloads.gaussian_cols(n, m, "inv_sq", seed, device=dev)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    err = metrics.rel_fro(to64(Y), sketch.sketch(op, to64(A)))
    say("  rel err", err)
    assert err <= TOL


def test_partial_split_bf16_plan_uses_fp32():
    dev = device()
    n, p, l, m = 4000, 4, 96, 130
    plan = bs.Plan(n, p, l, 8, precision=bs.SPLIT_BF16, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", 8, device=dev)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    assert metrics.rel_fro(to64(Y), sketch.sketch(rng.Plan(n, p, l, 8), to64(A))) <= TOL


def test_partial_equals_power_of_two_plan_on_padded_input():
    dev = device()
    n, p, l, m = 12000, 4, 300, 64
    r = n // p
    rp = 1 << (r - 1).bit_length()
    A = workloads.gaussian_cols(n, m, "inv_sq", 2, device=dev)
    Ap = torch.zeros(p * rp, m, device=dev)
    for i in range(p):
        Ap[i * rp:i * rp + r] = A[i * r:(i + 1) * r]
    Y = bs.bsrht_apply(bs.Plan(n, p, l, 6, device=dev), A)
    Yp = bs.bsrht_apply(bs.Plan(p * rp, p, l, 6, device=dev), Ap)
    torch.cuda.synchronize()
    assert metrics.rel_fro(to64(Y), to64(Yp)) < 2e-6


@pytest.mark.parametrize("n,p,l,m,lda_pad", [
    (1200, 4, 50, 19, 0),       # r = 300 -> 512: one chunk per block, partial
    (2800, 4, 300, 70, 3),      # r = 700 -> 1024: a full and a partial chunk; odd lda
    (800, 4, 77, 65, 0),        # r = 200 -> 256: 4-wave kernel (256-column chunks)
    (4000, 2, 600, 130, 0),     # r = 2000 -> 2048: 3 full + 1 partial chunk, two
                                # sample groups, a ragged second row tile
    (3074, 2, 40, 9, 1),        # r = 1537 -> 2048: odd block starts
    (400, 4, 30, 12, 0),        # r = 100 -> 128: direct evaluation
])
def test_partial_right_sketch(n, p, l, m, lda_pad):
    """Y = A Omega^T on padded plans: the streaming right-side kernel walks
    the chunks that hold columns of A (the last one of a block masked past
    r); blocks padded to fewer than 256 columns take the direct evaluation."""
    dev = device()
    say("partial right", n, p, l, m, lda_pad)
    plan = bs.Plan(n, p, l, 4, device=dev)
    A0 = workloads.gaussian_rows(m, n, "inv_sq", 4, device=dev)
    if lda_pad:
        big = torch.zeros(m, n + lda_pad, device=dev)
        big[:, :n] = A0
        A = big[:, :n]
    else:
        A = A0
    Y = bs.bsrht_apply_right(plan, A)
    Y2 = bs.bsrht_apply_right(plan, A)
    torch.cuda.synchronize()
    err = metrics.rel_fro(to64(Y), sketch.sketch_right(rng.Plan(n, p, l, 4), to64(A0)))
    say("  rel err", err)
    assert err <= TOL
    assert torch.equal(Y, Y2)


def test_partial_rsvd():
    dev = device()
    n, m, p, l, k = 6000, 200, 3, 64, 20   # r = 2000 -> 2048
    A = workloads.lowrank_tall(n, m, "inv_sq", 3, device=dev)
    plan = bs.Plan(n, p, l, 7, device=dev)
    U, S, V, info = bs.rsvd(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.lowrank_fro_error(Ah, to64(U), to64(S), to64(V))
    Uo, So, Vo = lowrank.rsvd(rng.Plan(n, p, l, 7), Ah, k)
    err_o = metrics.lowrank_fro_error(Ah, Uo, So, Vo)
    say("  partial rsvd err", err, "oracle", err_o)
    assert err <= 1.01 * err_o


@pytest.mark.parametrize("n,p,l,k", [
    (3000, 3, 128, 20),   # r = 1000 -> 1024: padded blocks in both sketches of Algorithm 2
    (2400, 4, 600, 40),   # r = 600 -> 1024: l > 512 (16-wave kernel); rank-512 A, so
                          # Omega A Omega^T is singular and Remark 3.1's split is taken
])
def test_partial_nystrom(n, p, l, k):
    dev = device()
    A = workloads.spd(n, 512, "inv_sq", 11, device=dev)
    plan = bs.Plan(n, p, l, 9, device=dev)
    U, lam, info = bs.nystrom(plan, A, k)
    torch.cuda.synchronize()
    Ah = to64(A)
    err = metrics.trace_error(Ah, to64(U), to64(lam))
    Uo, lo, fb = lowrank.nystrom(rng.Plan(n, p, l, 9), Ah, k)
    err_o = metrics.trace_error(Ah, Uo, lo)
    say("  partial nystrom err", err, "oracle", err_o, "info", int(info.item()),
        "oracle fallback", fb)
    assert err <= 1.01 * err_o


def test_partial_plan_rejected_by_batch():
    dev = device()
    plan = bs.Plan(300, 3, 20, 1, device=dev)
    A = torch.zeros(300, 64, device=dev)
    Y = torch.zeros(20, 64, device=dev)
    ws = torch.zeros(max(1, bs.bsrht_apply_workspace(plan, 64)), dtype=torch.uint8, device=dev)
    table = torch.zeros(bs.batch_table_bytes(), dtype=torch.uint8, device=dev)
    with pytest.raises(bs.BsrhtError):
        bs.apply_batch([(plan, A, Y, ws)], table)
