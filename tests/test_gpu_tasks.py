"""Non-blocking randomized SVD, Nystrom and single-view SVD (rsvd_start,
nystrom_start, nystrom_shifted_start, rsvd_single_view_start and
bsrht_task_poll / wait / destroy of include/bsrht.h; sections 3.1 to 3.3):
the same coroutines as the blocking
calls run with an asynchronous context, so on the same plan and input their
results must equal the blocking calls' bitwise, also with two tasks in
flight on two streams and with a task destroyed before it has finished."""
import time

import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from tests.gpu_util import device, say

pytestmark = pytest.mark.gpu


def _inputs(dev):
    A = workloads.lowrank_tall(8192, 300, "inv_sq", 3, device=dev)
    rplan = bs.Plan(8192, 8, 128, 5, device=dev)
    B = workloads.spd(2048, 512, "inv_sq", 11, device=dev)
    nplan = bs.Plan(2048, 4, 256, 12, device=dev)
    return A, rplan, B, nplan


def test_tasks_on_two_streams_equal_blocking_calls():
    dev = device()
    A, rplan, B, nplan = _inputs(dev)
    U0, S0, V0, i0 = bs.rsvd(rplan, A, 40)
    W0, L0, j0 = bs.nystrom(nplan, B, 32)
    X0, M0, k0 = bs.nystrom(nplan, B, 32, shifted=True)
    torch.cuda.synchronize()
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    t1, U1, S1, V1, i1 = bs.rsvd_start(rplan, A, 40, stream=s1)
    t2, W1, L1, j1 = bs.nystrom_start(nplan, B, 32, stream=s2)
    t3, X1, M1, k1 = bs.nystrom_start(nplan, B, 32, stream=s3, shifted=True)
    pending = {"rsvd": t1, "nystrom": t2, "nystrom_shifted": t3}
    polls = 0
    deadline = time.time() + 60.0
    while pending:
        assert time.time() < deadline, f"tasks still running: {sorted(pending)}"
        for name in list(pending):
            if pending[name].poll():
                del pending[name]
        polls += 1
    torch.cuda.synchronize()
    say("tasks finished after", polls, "poll rounds")
    for got, ref in [(U1, U0), (S1, S0), (V1, V0), (i1, i0), (W1, W0), (L1, L0), (j1, j0),
                     (X1, X0), (M1, M0), (k1, k0)]:
        assert torch.equal(got, ref)
    for t in (t1, t2, t3):
        t.close()


def test_task_wait_and_destroy_before_finish():
    dev = device()
    A, rplan, B, nplan = _inputs(dev)
    U0, S0, V0, i0 = bs.rsvd(rplan, A, 40)
    W0, L0, j0 = bs.nystrom(nplan, B, 32)
    torch.cuda.synchronize()
    t, U1, S1, V1, i1 = bs.rsvd_start(rplan, A, 40)
    t.wait()
    assert t.poll()
    t.close()
    t, W1, L1, j1 = bs.nystrom_start(nplan, B, 32)
    t.close()  # destroy waits for the unfinished task
    torch.cuda.synchronize()
    assert torch.equal(U1, U0) and torch.equal(S1, S0) and torch.equal(V1, V0)
    assert torch.equal(W1, W0) and torch.equal(L1, L0) and torch.equal(j1, j0)


def test_task_start_argument_errors():
    dev = device()
    A, rplan, B, nplan = _inputs(dev)
    with pytest.raises(bs.BsrhtError):
        bs.rsvd_start(rplan, A, 40, ws=torch.zeros(16, dtype=torch.uint8, device=dev))
    with pytest.raises(bs.BsrhtError):
        bs.nystrom_start(nplan, B, 0)


def _sv_plans(N1, N2, l, s, seed, dev):
    """Omega (l x N2), Gamma (l x N1), Phi (s x N1), Psi (s x N2)."""
    return [bs.Plan(N2, 4, l, seed, device=dev), bs.Plan(N1, 4, l, seed + 1, device=dev),
            bs.Plan(N1, 8, s, seed + 2, device=dev), bs.Plan(N2, 2, s, seed + 3, device=dev)]


def test_single_view_tasks_equal_blocking_calls():
    """rsvd_single_view_start on a full-rank input and on a rank-30 input with
    l = 64 (the bases then come from the eigen split, whose eigenvalues are
    read back mid-task), both in flight at once on two streams, against the
    blocking call."""
    dev = device()
    A = workloads.lowrank_tall(4096, 512, "inv_sq", 5, device=dev)
    rs = torch.Generator(device=dev).manual_seed(4)
    B = torch.randn(2048, 30, generator=rs, device=dev, dtype=torch.float64)
    C = torch.randn(30, 512, generator=rs, device=dev, dtype=torch.float64)
    R = (B @ C).float()
    pa = _sv_plans(4096, 512, 64, 128, 21, dev)
    pr = _sv_plans(2048, 512, 64, 128, 31, dev)
    ref_a = bs.rsvd_single_view(*pa, A, 30)
    ref_r = bs.rsvd_single_view(*pr, R, 30)
    torch.cuda.synchronize()
    assert int(ref_r[3].item()) & bs.INFO_QB_FALLBACK
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ta, *got_a = bs.rsvd_single_view_start(*pa, A, 30, stream=s1)
    tr, *got_r = bs.rsvd_single_view_start(*pr, R, 30, stream=s2)
    pending = {"full rank": ta, "rank 30": tr}
    deadline = time.time() + 60.0
    while pending:
        assert time.time() < deadline, f"tasks still running: {sorted(pending)}"
        for name in list(pending):
            if pending[name].poll():
                del pending[name]
    torch.cuda.synchronize()
    for got, ref in zip(got_a + got_r, list(ref_a) + list(ref_r)):
        assert torch.equal(got, ref)
    ta.close()
    tr.close()
    ws = torch.zeros(bs.rsvd_single_view_workspace(*pa, 30), dtype=torch.uint8, device=dev)
    with pytest.raises(bs.BsrhtError):  # Phi and Gamma swapped: inconsistent plans
        bs.rsvd_single_view_start(pa[0], pa[2], pa[1], pa[3], A, 30, ws=ws)
