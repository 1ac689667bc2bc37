"""Serving runtime on the GPU: a mix of sketch and randomized-SVD jobs run
concurrently through the server's stream slots gives, job by job, exactly the
result of the same library call made alone (every reduction runs in a fixed
order), and sampled small jobs match the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch, lowrank, metrics
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu


def _jobs(count, seed):
    rs = np.random.default_rng(seed)
    out = []
    for i in range(count):
        a = int(rs.integers(10, 15))
        n = 1 << a
        p = int(rs.choice([1, 2, 4, 16]))
        m = int(rs.integers(1, 300))
        k = int(rs.integers(1, 40))
        l = min(2 * k + 8, n)
        kind = bs.JOB_SKETCH if i % 3 == 0 else bs.JOB_RSVD
        prec = bs.SPLIT_BF16 if i % 5 == 0 else bs.FP32
        out.append(dict(id=i, kind=kind, n=n, m=m, p=p, l=l, k=k, prec=prec,
                        seed=int(rs.integers(0, 4)), data=int(rs.integers(0, 2 ** 31))))
    return out


def _payload(js, dev):
    A = workloads.gaussian_cols(js["n"], js["m"], "pow1.5", js["data"], device=dev)
    n, m, l, k = js["n"], js["m"], js["l"], js["k"]
    if js["kind"] == bs.JOB_SKETCH:
        return A, dict(Y=torch.full((l, m), float("nan"), device=dev))
    return A, dict(U=torch.full((n, k), float("nan"), device=dev),
                   S=torch.full((k,), float("nan"), dtype=torch.float64, device=dev),
                   V=torch.full((m, k), float("nan"), device=dev),
                   info=torch.zeros(1, dtype=torch.int32, device=dev))


def _desc(js, A, out):
    pa = (js["n"], js["p"], js["l"], js["seed"], bs.WITH_REPLACEMENT, js["prec"])
    if js["kind"] == bs.JOB_SKETCH:
        return bs.sketch_job(js["id"], pa, A, out["Y"])
    return bs.rsvd_job(js["id"], pa, A, js["k"], out["U"], out["S"], out["V"], out["info"])


def _alone(js, A):
    plan = bs.Plan(js["n"], js["p"], js["l"], js["seed"], precision=js["prec"], device=A.device)
    if js["kind"] == bs.JOB_SKETCH:
        return dict(Y=bs.bsrht_apply(plan, A))
    U, S, V, info = bs.rsvd(plan, A, js["k"])
    return dict(U=U, S=S, V=V, info=info)


def test_mix_equals_alone_and_matches_oracle():
    dev = device()
    jobs = _jobs(120, 5)
    arena = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    payloads = {}
    with bs.Server(arena=arena, workers=4) as srv:
        for js in jobs:
            A, out = _payload(js, dev)
            torch.cuda.synchronize()
            payloads[js["id"]] = (A, out)
            srv.submit(_desc(js, A, out))
        srv.drain()
        res = {r.id: r for r in srv.poll(1000)}
        st = srv.stats()
    say("stats", st)
    assert len(res) == len(jobs)
    assert all(r.status == 0 for r in res.values())
    assert st["peak_running"] >= 2          # jobs really overlapped
    for js in jobs:
        A, out = payloads[js["id"]]
        ref = _alone(js, A)
        torch.cuda.synchronize()
        for name, t in ref.items():
            assert torch.equal(out[name], t), (js, name)
    # oracle parity on a sample of the small jobs
    checked = 0
    for js in jobs:
        if js["n"] > 4096 or checked >= 8:
            continue
        A, out = payloads[js["id"]]
        op = rng.Plan(js["n"], js["p"], js["l"], js["seed"])
        tol = 1e-4 if js["prec"] == bs.SPLIT_BF16 else 1e-5
        if js["kind"] == bs.JOB_SKETCH:
            err = metrics.rel_fro(to64(out["Y"]), sketch.sketch(op, to64(A)))
            assert err <= tol, (js, err)
        else:
            Ah = to64(A)
            err = metrics.lowrank_fro_error(Ah, to64(out["U"]), to64(out["S"]), to64(out["V"]))
            Uo, So, Vo = lowrank.rsvd(op, Ah, js["k"])
            err_o = metrics.lowrank_fro_error(Ah, Uo, So, Vo)
            if js["k"] >= min(js["n"], js["m"]):
                # exact recovery: the oracle's error is FP64 rounding, the
                # GPU's the FP32 floor
                assert err < 1e-5, (js, err, err_o)
            else:
                assert err <= 1.01 * err_o, (js, err, err_o)
        checked += 1
    assert checked >= 4


def test_small_sketch_jobs_run_batched_and_equal_alone():
    """A burst of small FP32 sketch jobs (with a few RSVD and split-BF16 jobs
    between them) on two slots: the small sketches run as batched launches
    (one persistent, graph-replayed launch per batch), and every job's result
    is bitwise the single call's."""
    dev = device()
    rs = np.random.default_rng(11)
    jobs = []
    for i in range(90):
        n = 1 << int(rs.integers(10, 15))
        p = int(rs.choice([1, 4, 16]))
        m = int(rs.integers(1, 200))
        k = int(rs.integers(1, 20))
        kind = bs.JOB_RSVD if i % 15 == 7 else bs.JOB_SKETCH
        prec = bs.SPLIT_BF16 if i % 11 == 3 else bs.FP32
        l = min(int(rs.choice([32, 100, 300, 700])), n) if kind == bs.JOB_SKETCH else 2 * k + 8
        jobs.append(dict(id=i, kind=kind, n=n, m=m, p=p, l=l, k=k, prec=prec,
                         seed=int(rs.integers(0, 3)), data=int(rs.integers(0, 2 ** 31))))
    arena = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    payloads = {js["id"]: _payload(js, dev) for js in jobs}
    torch.cuda.synchronize()
    with bs.Server(arena=arena, workers=2) as srv:
        for js in jobs:
            A, out = payloads[js["id"]]
            srv.submit(_desc(js, A, out))
        srv.drain()
        res = {r.id: r for r in srv.poll(1000)}
        st = srv.stats()
    say("stats", st)
    assert len(res) == len(jobs) and all(r.status == 0 for r in res.values())
    assert st["batches"] >= 1 and st["batched_jobs"] >= 2 * st["batches"]
    for js in jobs:
        A, out = payloads[js["id"]]
        ref = _alone(js, A)
        torch.cuda.synchronize()
        for name, t in ref.items():
            assert torch.equal(out[name], t), (js, name)


def _nys_jobs(count, seed):
    """Sketch, RSVD and Nystrom jobs in turn; Nystrom payloads are full-rank
    SPD n x n matrices (n = 2^9 .. 2^11), so no oracle comparison below can
    pass by exact recovery."""
    rs = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = (bs.JOB_SKETCH, bs.JOB_RSVD, bs.JOB_NYSTROM)[i % 3]
        n = 1 << int(rs.integers(9, 12) if kind == bs.JOB_NYSTROM else rs.integers(10, 14))
        p = int(rs.choice([1, 2, 4, 16]))
        m = n if kind == bs.JOB_NYSTROM else int(rs.integers(1, 300))
        k = int(rs.integers(4, 40))
        l = min(2 * k + 8, n)
        prec = bs.SPLIT_BF16 if i % 7 == 2 else bs.FP32
        out.append(dict(id=i, kind=kind, n=n, m=m, p=p, l=l, k=k, prec=prec,
                        seed=int(rs.integers(0, 4)), data=int(rs.integers(0, 2 ** 31))))
    return out


def _nys_payload(js, dev):
    if js["kind"] != bs.JOB_NYSTROM:
        return _payload(js, dev)
    n, k = js["n"], js["k"]
    A = workloads.spd(n, n, "inv_sq", js["data"], device=dev)
    return A, dict(U=torch.full((n, k), float("nan"), device=dev),
                   lam=torch.full((k,), float("nan"), dtype=torch.float64, device=dev),
                   info=torch.zeros(1, dtype=torch.int32, device=dev))


def test_nystrom_jobs_in_mix_equal_alone_and_match_oracle():
    """Nystrom jobs (section 3.2, Algorithm 2) served next to sketch and RSVD
    jobs on four slots: each result is bitwise the stand-alone nystrom call's,
    and sampled jobs are within 1% of the FP64 oracle's trace error with the
    same Omega."""
    dev = device()
    jobs = _nys_jobs(60, 17)
    arena = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    payloads = {js["id"]: _nys_payload(js, dev) for js in jobs}
    torch.cuda.synchronize()
    with bs.Server(arena=arena, workers=4) as srv:
        for js in jobs:
            A, out = payloads[js["id"]]
            pa = (js["n"], js["p"], js["l"], js["seed"], bs.WITH_REPLACEMENT, js["prec"])
            if js["kind"] == bs.JOB_NYSTROM:
                srv.submit(bs.nystrom_job(js["id"], pa, A, js["k"], out["U"], out["lam"],
                                          out["info"]))
            else:
                srv.submit(_desc(js, A, out))
        srv.drain()
        res = {r.id: r for r in srv.poll(1000)}
        st = srv.stats()
    say("stats", st)
    assert len(res) == len(jobs) and all(r.status == 0 for r in res.values())
    assert st["peak_running"] >= 2
    checked = 0
    for js in jobs:
        A, out = payloads[js["id"]]
        if js["kind"] != bs.JOB_NYSTROM:
            ref = _alone(js, A)
        else:
            plan = bs.Plan(js["n"], js["p"], js["l"], js["seed"], precision=js["prec"],
                           device=dev)
            U, lam, info = bs.nystrom(plan, A, js["k"])
            ref = dict(U=U, lam=lam, info=info)
        torch.cuda.synchronize()
        for name, t in ref.items():
            assert torch.equal(out[name], t), (js, name)
        if js["kind"] == bs.JOB_NYSTROM and checked < 8:
            Ah = to64(A)
            err = metrics.trace_error(Ah, to64(out["U"]), to64(out["lam"]))
            Uo, lo, fb = lowrank.nystrom(rng.Plan(js["n"], js["p"], js["l"], js["seed"]), Ah,
                                         js["k"])
            err_o = metrics.trace_error(Ah, Uo, lo)
            say("  nystrom job", js["id"], js["n"], js["p"], js["l"], js["k"], "err", err,
                "oracle", err_o)
            assert err <= 1.01 * err_o, (js, err, err_o)
            checked += 1
    assert checked >= 6
