"""GPU parity of the block SRHT sketch (section 2, eq. (2.3)-(2.4)) against the
FP64 oracle, through the C ABI.

Tables (R, D, Dt) must match the oracle bit for bit; the FP32 sketch must be
within 1e-5 relative Frobenius error of the FP64 oracle on the same input.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch, metrics
from tests.gpu_util import device, to64, unpack_bits, say

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _tables_match(plan, op):
    R, Db, Dtb = plan.export()
    assert np.array_equal(R.astype(np.int64), op.R)
    assert np.array_equal(unpack_bits(Db, op.n), op.D_bits.ravel())
    lw = (op.l + 31) // 32
    dt = np.stack([unpack_bits(Dtb[i * lw:(i + 1) * lw], op.l) for i in range(op.p)])
    assert np.array_equal(dt, op.Dt_bits)


@pytest.mark.parametrize("name", sorted(f[:-5] for f in os.listdir(GOLDEN) if f.endswith(".json")))
def test_tables_match_golden(name):
    dev = device()
    doc = json.load(open(os.path.join(GOLDEN, name + ".json")))
    say("golden", name)
    plan = bs.Plan(doc["n"], doc["p"], doc["l"], doc["seed"], doc["sampling"], device=dev)
    R, Db, Dtb = plan.export()
    assert R.tolist() == doc["R"]
    assert Db.tolist() == doc["Dbits"]
    assert Dtb.tolist() == doc["Dtbits"]
    if "omega" in doc:
        # Omega columns = sketch of the identity
        n = doc["n"]
        I = torch.eye(n, dtype=torch.float32, device=dev)
        Om = bs.bsrht_apply(plan, I)
        torch.cuda.synchronize()
        assert np.max(np.abs(to64(Om) - np.array(doc["omega"]))) < 1e-6


TABLE_CASES = [
    (1 << 20, 16, 512, 0, rng.WITH_REPLACEMENT),
    (65536, 64, 1024, 7, rng.WITH_REPLACEMENT),
    (4096, 1, 4096, 3, rng.WITHOUT_REPLACEMENT),
    (1 << 16, 1, 700, 5, rng.WITHOUT_REPLACEMENT),
    (96, 96, 33, 2 ** 64 - 1, rng.WITH_REPLACEMENT),
    (48, 3, 17, 11, rng.WITH_REPLACEMENT),
]


@pytest.mark.parametrize("n,p,l,seed,mode", TABLE_CASES)
def test_tables_bit_exact(n, p, l, seed, mode):
    dev = device()
    say("tables", n, p, l, seed, mode)
    _tables_match(bs.Plan(n, p, l, seed, mode, device=dev), rng.Plan(n, p, l, seed, mode))


def _align256(x):
    return (x + 255) // 256 * 256


def _round_robin_order(key):
    """A gather lane order the plan stores: per group of 1024 samples, the
    samples taken round-robin over key_j in 0..15 (round k holds the k-th
    sample, in draw order, of each key value that has one)."""
    out = []
    for g0 in range(0, len(key), 1024):
        rho = key[g0:g0 + 1024]
        buckets = [list(np.nonzero(rho == v)[0] + g0) for v in range(16)]
        for k in range(max(len(b) for b in buckets)):
            out += [b[k] for b in buckets if k < len(b)]
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("n,p,l,seed,mode", TABLE_CASES + [(10_000_000, 16, 2000, 0, 0)])
def test_gather_lane_order(n, p, l, seed, mode):
    """The two lane order regions of the plan tables (after R, D and Dt) are
    permutations of the samples within each 1024-sample group, equal to the
    round-robin orders over R_j mod 16 (column kernels) and (R_j >> 2) mod 16
    (right-side kernel)."""
    dev = device()
    say("lane order", n, p, l, seed, mode)
    plan = bs.Plan(n, p, l, seed, mode, device=dev)
    R = plan.export()[0].astype(np.int64)
    off = (_align256(4 * l) + _align256(4 * ((p * plan.rp + 31) // 32))
           + _align256(4 * p * ((l + 31) // 32)))
    for shift in (0, 2):
        order = plan.tables[off:off + 4 * l].view(torch.int32).cpu().numpy().astype(np.int64)
        for g0 in range(0, l, 1024):
            assert sorted(order[g0:g0 + 1024].tolist()) == list(range(g0, min(l, g0 + 1024)))
        assert np.array_equal(order, _round_robin_order((R >> shift) & 15))
        off += _align256(4 * l)


@pytest.mark.parametrize("n,p,l,m,precision,right", [
    (1 << 16, 16, 512, 200, bs.FP32, False),        # 8-wave kernel
    (1 << 16, 16, 1000, 130, bs.FP32, False),       # 16-wave kernel
    (1 << 16, 16, 512, 200, bs.SPLIT_BF16, False),  # split-BF16, 8 waves
    (1 << 16, 16, 1000, 70, bs.SPLIT_BF16, False),  # split-BF16, 16 waves
    (1 << 16, 16, 512, 100, bs.FP32, True),         # right-side, b = 512
    (1 << 14, 64, 300, 65, bs.FP32, True),          # right-side, b = 256
])
def test_lane_order_leaves_results_bitwise_unchanged(n, p, l, m, precision, right):
    """The gather lane orders only assign samples to lanes: with both order
    regions overwritten by the identity (draw order), every sketch is
    bitwise the same."""
    dev = device()
    say("lane order identity", n, p, l, m, precision, right)
    plan = bs.Plan(n, p, l, 17, bs.WITH_REPLACEMENT, precision, device=dev)
    if right:
        A = workloads.gaussian_rows(m, n, "inv_sq", 17, device=dev)
        run = lambda: bs.bsrht_apply_right(plan, A).clone()
    else:
        A = workloads.gaussian_cols(n, m, "inv_sq", 17, device=dev)
        run = lambda: bs.bsrht_apply(plan, A).clone()
    Y1 = run()
    off = (_align256(4 * l) + _align256(4 * ((p * plan.rp + 31) // 32))
           + _align256(4 * p * ((l + 31) // 32)))
    ident = torch.arange(l, dtype=torch.int32, device=dev)
    for k in range(2):
        o = off + k * _align256(4 * l)
        plan.tables[o:o + 4 * l].view(torch.int32).copy_(ident)
    Y2 = run()
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


SKETCH_CASES = [
    # n, p, l, m, mode   -- spans chunk sizes 64..512, ragged column tiles,
    # several row splits and sample groups, r = 1 .. 2^14, l > r
    (4096, 4, 128, 256, 0),       # the small RSVD workload's shape
    (4096, 4, 128, 100, 0),       # ragged column tile
    (8192, 8, 300, 65, 0),        # r = 1024, l not a multiple of 64
    (16384, 1, 513, 33, 0),       # r = 2^14, l = 513: 16-wave kernel
    (2048, 8, 1100, 7, 0),        # r = 256 < l: 16-wave kernel, two sample groups
    (1024, 8, 200, 64, 0),        # r = 128 (chunk 128)
    (1024, 16, 77, 130, 0),       # r = 64 (smallest fused chunk)
    (512, 16, 40, 5, 0),          # r = 32: direct kernel
    (64, 64, 20, 9, 0),           # r = 1: Rademacher
    (4096, 2, 1024, 31, 1),       # without replacement
    (2048, 1, 2048, 16, 1),       # p = 1, l = r = n: orthogonal
    (4096, 4, 1, 40, 0),          # l = 1
    (4096, 4, 128, 1, 0),         # m = 1
]


@pytest.mark.parametrize("n,p,l,m,mode", SKETCH_CASES)
def test_sketch_parity(n, p, l, m, mode):
    dev = device()
    say("sketch", n, p, l, m, mode)
    seed = 1000 + n + p + l + m
    plan = bs.Plan(n, p, l, seed, mode, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", seed, device=dev)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    Y_ref = sketch.sketch(rng.Plan(n, p, l, seed, mode), to64(A))
    err = metrics.rel_fro(to64(Y), Y_ref)
    say("  rel err", err)
    assert err <= TOL_FP32


def test_strided_input_and_output():
    dev = device()
    n, p, l, m = 4096, 4, 96, 70
    plan = bs.Plan(n, p, l, 4, device=dev)
    big = workloads.gaussian_cols(n, 200, "inv_sq", 5, device=dev)
    A = big[:, 13:13 + m]                 # lda = 200, offset start
    Ybig = torch.full((l, 150), 7.0, device=dev)
    Y = Ybig[:, 20:20 + m]
    bs.bsrht_apply(plan, A, Y)
    torch.cuda.synchronize()
    Y_ref = sketch.sketch(rng.Plan(n, p, l, 4), to64(A))
    assert metrics.rel_fro(to64(Y), Y_ref) <= TOL_FP32
    assert torch.all(Ybig[:, :20] == 7.0) and torch.all(Ybig[:, 20 + m:] == 7.0)


def test_bitwise_repeatable():
    dev = device()
    n, p, l, m = 1 << 16, 16, 512, 256
    plan = bs.Plan(n, p, l, 9, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", 9, device=dev)
    Y1 = bs.bsrht_apply(plan, A).clone()
    Y2 = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)


def test_block_sum_identity():
    """Eq. (2.4): the sketch equals the sum of single-block sketches; and a p = 1
    plan on the first block's rows reproduces block 0 (subsample keying)."""
    dev = device()
    n, p, l, m = 8192, 4, 64, 48
    r = n // p
    plan = bs.Plan(n, p, l, 21, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", 21, device=dev)
    Y = bs.bsrht_apply(plan, A)
    parts = []
    for i in range(p):
        Ai = torch.zeros_like(A)
        Ai[i * r:(i + 1) * r] = A[i * r:(i + 1) * r]
        parts.append(bs.bsrht_apply(plan, Ai))
    sub = bs.bsrht_apply(bs.Plan(r, 1, l, 21, device=dev), A[:r].contiguous())
    torch.cuda.synchronize()
    assert metrics.rel_fro(to64(sum(parts)), to64(Y)) < 3e-6
    assert metrics.rel_fro(to64(sub), to64(parts[0])) < 3e-6


def test_errors_and_empty():
    dev = device()
    plan = bs.Plan(4096, 4, 64, 1, device=dev)
    L = bs.lib()
    A = torch.zeros(4096, 8, device=dev)
    Y = torch.zeros(64, 8, device=dev)
    ws = torch.zeros(1, dtype=torch.uint8, device=dev)
    assert L.bsrht_apply(plan.handle, bs._ptr(A), 0, 8, bs._ptr(Y), 8, None, 0, None) == 0
    assert L.bsrht_apply(plan.handle, bs._ptr(A), 8, 4, bs._ptr(Y), 8, None, 0, None) == -1
    assert L.bsrht_apply(plan.handle, bs._ptr(A), 8, 8, bs._ptr(Y), 7, None, 0, None) == -1
    assert L.bsrht_apply(plan.handle, None, 8, 8, bs._ptr(Y), 8, None, 0, None) == -1
    need = L.bsrht_apply_workspace(plan.handle, 8)
    if need > 0:
        assert L.bsrht_apply(plan.handle, bs._ptr(A), 8, 8, bs._ptr(Y), 8, bs._ptr(ws), 0,
                             None) == -2
    with pytest.raises(ValueError):
        bs.bsrht_apply(plan, torch.zeros(100, 8, device=dev))
