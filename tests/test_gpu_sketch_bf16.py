"""GPU parity of the split-BF16 matrix-core sketch against the FP64 oracle,
through the C ABI.

The block SRHT of section 2 (eq. (2.3)-(2.4)) with the H_16 Kronecker factor
on BF16 matrix cores and A split into BF16 hi + lo parts must stay within
1e-4 relative Frobenius error of the FP64 oracle (a single split loses at
most 2^-16 relative per element; a BF16-only input would be off by ~2^-9).
"""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch, metrics
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu

TOL_BF16 = 1e-4


def _bf16_launches(fn):
    """Run fn with the split-BF16 kernel timing hook on; return launch count."""
    bs.timing_enable(bs.TIMING_APPLY_BF16)
    try:
        fn()
        torch.cuda.synchronize()
        _, launches = bs.timing_read()
    finally:
        bs.timing_enable(bs.TIMING_OFF)
    return launches


CASES = [
    # n, p, l, m, mode -- chunk sizes 128 / 256 / 512, ragged column tiles,
    # row splits, several sample groups, l > r, and r < 128 (FP32 kernels)
    (4096, 4, 128, 256, 0),       # r = 1024, chunk 512
    (4096, 4, 128, 100, 0),       # ragged column tile (100 = 64 + 36)
    (8192, 8, 300, 65, 0),        # one column past a tile
    (16384, 1, 513, 33, 0),       # r = 2^14, l = 513: 16-wave kernel, only a ragged tile
    (2048, 8, 1100, 7, 0),        # r = 256 < l: 16-wave kernel, two sample groups
    (1024, 8, 200, 64, 0),        # r = 128 (chunk 128)
    (1 << 16, 1, 512, 130, 0),    # r = 2^16 as one block, ragged
    (4096, 2, 1024, 31, 1),       # without replacement
    (2048, 1, 2048, 16, 1),       # p = 1, l = r = n
    (4096, 4, 1, 40, 0),          # l = 1
    (4096, 4, 128, 1, 0),         # m = 1
    (1024, 16, 77, 130, 0),       # r = 64: below the matrix-core chunk
]


@pytest.mark.parametrize("n,p,l,m,mode", CASES)
def test_split_bf16_parity(n, p, l, m, mode):
    dev = device()
    say("split-bf16", n, p, l, m, mode)
    seed = 2000 + n + p + l + m
    plan = bs.Plan(n, p, l, seed, mode, precision=bs.SPLIT_BF16, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", seed, device=dev)
    out = {}
    launches = _bf16_launches(lambda: out.setdefault("Y", bs.bsrht_apply(plan, A)))
    if n // p >= 128:
        assert launches >= 1  # the matrix-core kernel ran
    else:
        assert launches == 0  # r < 128 runs the FP32 kernels
    Y_ref = sketch.sketch(rng.Plan(n, p, l, seed, mode), to64(A))
    err = metrics.rel_fro(to64(out["Y"]), Y_ref)
    say("  rel err", err)
    assert err <= TOL_BF16


def test_split_bf16_needs_low_part():
    """Entries 1 + k 2^-12 are exact in FP32 but not in BF16: dropping the lo
    part would cost ~1e-3 relative; the split keeps the result within 1e-5."""
    dev = device()
    n, p, l, m = 8192, 8, 256, 64
    k = torch.arange(n * m, device=dev, dtype=torch.float32).reshape(n, m) % 97
    A = 1.0 + k * 2.0 ** -12
    plan = bs.Plan(n, p, l, 77, precision=bs.SPLIT_BF16, device=dev)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    Y_ref = sketch.sketch(rng.Plan(n, p, l, 77), to64(A))
    err = metrics.rel_fro(to64(Y), Y_ref)
    say("  rel err", err)
    assert err <= 1e-5


def test_split_bf16_strided_and_repeatable():
    dev = device()
    n, p, l, m = 4096, 4, 96, 70
    plan = bs.Plan(n, p, l, 4, precision=bs.SPLIT_BF16, device=dev)
    big = workloads.gaussian_cols(n, 200, "inv_sq", 5, device=dev)
    A = big[:, 13:13 + m]                 # lda = 200, offset start
    Ybig = torch.full((l, 150), 7.0, device=dev)
    Y = Ybig[:, 20:20 + m]
    bs.bsrht_apply(plan, A, Y)
    Y2 = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    Y_ref = sketch.sketch(rng.Plan(n, p, l, 4), to64(A))
    assert metrics.rel_fro(to64(Y), Y_ref) <= TOL_BF16
    assert torch.equal(Y, Y2)
    assert torch.all(Ybig[:, :20] == 7.0) and torch.all(Ybig[:, 20 + m:] == 7.0)


def test_split_bf16_agrees_with_fp32_kernel():
    """Both precisions of the same plan agree to the split-BF16 tolerance."""
    dev = device()
    n, p, l, m = 1 << 16, 16, 512, 256
    A = workloads.gaussian_cols(n, m, "inv_sq", 9, device=dev)
    Yb = bs.bsrht_apply(bs.Plan(n, p, l, 9, precision=bs.SPLIT_BF16, device=dev), A)
    Yf = bs.bsrht_apply(bs.Plan(n, p, l, 9, device=dev), A)
    torch.cuda.synchronize()
    assert metrics.rel_fro(to64(Yb), to64(Yf)) <= TOL_BF16
