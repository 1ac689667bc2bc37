"""GPU parity of the batched sketch launch (bsrht_apply_batch) through the C ABI.

Each item of a batch must be bitwise the result of bsrht_apply on the same
arguments: the persistent kernels run the same workgroup tiles (same
template instance, chunk ranges and row splits) and the same fixed-order sum
of the split partials.  The launch is a graph captured on the first call for
a table and replayed afterwards with new descriptors, so the tests replay it
several times with different batches, with eager work and synchronisation in
between, and check every replay.
"""
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch, metrics
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu

# n, p, l, m: every 8-wave chunk size (r = 1024 -> 512-row chunks, 256 ->
# 256, 128 -> 128, 64 -> 64), the 16-wave kernel (l > 512, r >= 256), one and
# several row splits, ragged column tiles
SHAPES = [
    (4096, 4, 128, 256),
    (2048, 16, 77, 130),
    (8192, 8, 300, 65),
    (4096, 16, 600, 40),
    (65536, 4, 64, 96),
    (1024, 4, 64, 33),
    (1024, 16, 32, 20),
    (16384, 16, 1000, 7),
]


def _case(i, n, p, l, m, dev):
    plan = bs.Plan(n, p, l, 100 + i, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", 200 + i, device=dev)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8, device=dev)
    Y = torch.full((l, m), float("nan"), device=dev)
    ref = bs.bsrht_apply(plan, A)
    return plan, A, Y, ws, ref


def test_batch_bitwise_equals_single_calls():
    dev = device()
    cases = [_case(i, *s, dev) for i, s in enumerate(SHAPES)]
    table = torch.empty(bs.batch_table_bytes(), dtype=torch.uint8, device=dev)
    say("batch of", len(cases))
    bs.apply_batch([(c[0], c[1], c[2], c[3]) for c in cases], table)
    torch.cuda.synchronize()
    for (plan, A, Y, ws, ref), shp in zip(cases, SHAPES):
        say("  shape", shp)
        assert torch.equal(Y, ref)


def test_batch_graph_replays_with_new_descriptors():
    dev = device()
    cases = [_case(i, *s, dev) for i, s in enumerate(SHAPES)]
    table = torch.empty(bs.batch_table_bytes(), dtype=torch.uint8, device=dev)
    subsets = [[0, 2, 4], [1, 3, 5, 6, 7], [0, 1, 2, 3, 4, 5, 6, 7], [6], [2, 4]]
    junk = torch.randn(1 << 20, device=dev)
    for rep, sub in enumerate(subsets):
        for k in sub:
            cases[k][2].fill_(float("nan"))
        torch.cuda.synchronize()
        bs.apply_batch([(cases[k][0], cases[k][1], cases[k][2], cases[k][3]) for k in sub],
                       table)
        junk.mul_(1.0001)  # eager work between replays
        torch.cuda.synchronize()
        say("replay", rep, "items", sub)
        for k in sub:
            assert torch.equal(cases[k][2], cases[k][4]), (rep, k)


def test_batch_on_a_side_stream_matches_oracle():
    dev = device()
    n, p, l, m = 4096, 4, 96, 70
    plan = bs.Plan(n, p, l, 5, device=dev)
    A = workloads.gaussian_cols(n, m, "inv_sq", 6, device=dev)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8, device=dev)
    Y = torch.empty(l, m, device=dev)
    table = torch.empty(bs.batch_table_bytes(), dtype=torch.uint8, device=dev)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bs.apply_batch([(plan, A, Y, ws)], table, stream=side)
    side.synchronize()
    Y_ref = sketch.sketch(rng.Plan(n, p, l, 5), to64(A))
    assert metrics.rel_fro(to64(Y), Y_ref) <= 1e-5


def test_batch_rejections():
    dev = device()
    table = torch.empty(bs.batch_table_bytes(), dtype=torch.uint8, device=dev)
    ok = _case(0, 4096, 4, 128, 64, dev)
    item = (ok[0], ok[1], ok[2], ok[3])
    # a split-BF16 plan and blocks shorter than 64 rows take bsrht_apply
    pb = bs.Plan(4096, 4, 128, 1, precision=bs.SPLIT_BF16, device=dev)
    with pytest.raises(bs.BsrhtError) as e:
        bs.apply_batch([item, (pb, ok[1], ok[2], ok[3])], table)
    assert e.value.status == -4
    ps = bs.Plan(1024, 32, 16, 1, device=dev)  # r = 32
    As = workloads.gaussian_cols(1024, 8, "inv_sq", 1, device=dev)
    Ys = torch.empty(16, 8, device=dev)
    with pytest.raises(bs.BsrhtError) as e:
        bs.apply_batch([(ps, As, Ys, None)], table)
    assert e.value.status == -4
    # too many items, too small a table, a short workspace
    with pytest.raises(bs.BsrhtError) as e:
        bs.apply_batch([item] * (bs.BATCH_MAX + 1), table)
    assert e.value.status == -1
    with pytest.raises(bs.BsrhtError) as e:
        bs.apply_batch([item], table[:16])
    assert e.value.status == -1
    big = _case(1, 65536, 4, 64, 96, dev)
    if bs.bsrht_apply_workspace(big[0], 96) > 0:
        with pytest.raises(bs.BsrhtError) as e:
            bs.apply_batch([(big[0], big[1], big[2], None)], table)
        assert e.value.status == -2
    torch.cuda.synchronize()
