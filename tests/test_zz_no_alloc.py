"""The allocation-free sketch entry point (bsrht_apply_noalloc) through the C
ABI: on two calls in a row, the second with a smaller input, its result is
bitwise that of bsrht_apply with a caller workspace (same kernels, launch
decomposition and summation order), in FP32 and split-BF16; a call whose
partials would exceed the library's scratch array is rejected before
anything is enqueued and leaves its output untouched."""
import ctypes

import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from tests.gpu_util import device, say

pytestmark = pytest.mark.gpu


def _noalloc(plan, A, Y):
    L = bs.lib()
    m = A.shape[1]
    return L.bsrht_apply_noalloc(plan.handle, ctypes.c_void_p(A.data_ptr()), m, A.stride(0),
                                 ctypes.c_void_p(Y.data_ptr()), Y.stride(0),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("precision", [bs.FP32, bs.SPLIT_BF16], ids=["fp32", "split_bf16"])
def test_noalloc_equals_apply_on_two_calls(precision):
    dev = device()
    # first call: 2^18 x 1024, p = 4, l = 512 (16 row splits: 32 MiB of partials);
    # second: 2^14 x 100, p = 2, l = 200 (fewer, smaller partials)
    cases = [(1 << 18, 1024, 4, 512, 3), (1 << 14, 100, 2, 200, 4)]
    outs = []
    for n, m, p, l, seed in cases:
        plan = bs.Plan(n, p, l, seed, precision=precision, device=dev)
        need = bs.bsrht_apply_workspace(plan, m)
        say("noalloc", n, m, p, l, "partials bytes", need)
        assert 0 < need <= bs.NOALLOC_SCRATCH_BYTES
        A = workloads.gaussian_cols(n, m, "inv_sq", seed, device=dev)
        Y = torch.full((l, m), float("nan"), device=dev)
        assert _noalloc(plan, A, Y) == 0
        outs.append((plan, A, Y))
    torch.cuda.synchronize()
    for plan, A, Y in outs:
        ref = bs.bsrht_apply(plan, A)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)


def test_noalloc_rejects_partials_beyond_the_scratch():
    dev = device()
    n, p, l, m = 1 << 20, 16, 1024, 64   # 16-wave kernel, 256 row splits: 64 MiB of partials
    plan = bs.Plan(n, p, l, 5, device=dev)
    need = bs.bsrht_apply_workspace(plan, m)
    say("noalloc reject: partials bytes", need)
    assert need > bs.NOALLOC_SCRATCH_BYTES
    A = torch.zeros(n, m, device=dev)
    Y = torch.full((l, m), 7.0, device=dev)
    assert _noalloc(plan, A, Y) == -2     # BSRHT_ENOMEM, nothing enqueued
    torch.cuda.synchronize()
    assert torch.all(Y == 7.0)
    # and the entry point still works afterwards on a smaller input
    plan2 = bs.Plan(1 << 16, 4, 256, 6, device=dev)
    A2 = workloads.gaussian_cols(1 << 16, 300, "inv_sq", 6, device=dev)
    Y2 = torch.empty(256, 300, device=dev)
    assert _noalloc(plan2, A2, Y2) == 0
    torch.cuda.synchronize()
    assert torch.equal(Y2, bs.bsrht_apply(plan2, A2))
