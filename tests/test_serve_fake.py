"""Serving scheduler on the host-only executor (no GPU): admission against the
byte budget, arrival-order admission with bounded backfill, the plan cache,
concurrency limits and thread-safe submission.  The fake executor runs a job
by sleeping in proportion to its input bytes; the scheduler, the arena
allocator and the cache are the same code that drives the GPU."""
import threading
import time

import pytest

import paper_2210_11295_amd as bs


def job(i, n=1 << 14, m=64, p=4, l=64, k=16, seed=1, kind=bs.JOB_RSVD):
    return bs.JobDesc(id=i, kind=kind, n=n, m=m, p=p, l=l, k=k, seed=seed,
                      sampling=bs.WITH_REPLACEMENT, precision=bs.FP32, lda=m, ldy=m)


def run_all(srv, jobs):
    for j in jobs:
        srv.submit(j)
    srv.drain()
    res = srv.poll(max_results=len(jobs) + 8)
    assert len(res) == len(jobs)
    return res


def test_every_job_completes_with_ordered_timestamps():
    with bs.Server(fake_bytes=1 << 30, workers=3, seconds_per_gb=0.5) as srv:
        res = run_all(srv, [job(i, seed=i % 3) for i in range(40)])
        assert sorted(r.id for r in res) == list(range(40))
        for r in res:
            assert r.status == 0
            assert r.t_submit <= r.t_start <= r.t_done
            assert r.arena_bytes > 0
        st = srv.stats()
        assert st["submitted"] == st["completed"] == 40
        assert st["queued"] == 0
        assert 1 <= st["peak_running"] <= 3


def test_budget_is_never_exceeded_and_limits_concurrency():
    one = bs.bsrht_job_bytes(job(0))
    assert one > 0
    budget = int(2.5 * one)      # room for two jobs at a time (plan tables shared)
    with bs.Server(fake_bytes=budget, workers=6, seconds_per_gb=2.0) as srv:
        run_all(srv, [job(i) for i in range(12)])
        st = srv.stats()
        assert st["peak_arena_bytes"] <= budget
        assert st["peak_running"] == 2
        assert st["plan_misses"] == 1 and st["plan_hits"] == 11


def test_concurrency_shortens_the_makespan():
    jobs = [job(i) for i in range(8)]
    t = 4 * (1 << 14) * 64 / 1e9 * 20.0     # seconds per job at 20 s/GB
    with bs.Server(fake_bytes=1 << 30, workers=4, seconds_per_gb=20.0) as srv:
        t0 = srv.clock()
        res = run_all(srv, jobs)
        span = max(r.t_done for r in res) - t0
    assert span < 8 * t * 0.6          # serial would take 8 t
    assert span >= 2 * t * 0.9         # 8 jobs on 4 workers: at least 2 rounds


def test_rejections():
    with bs.Server(fake_bytes=1 << 20, workers=2) as srv:
        big = job(1, n=1 << 20, m=2048, l=544, k=256)
        with pytest.raises(bs.BsrhtError) as e:
            srv.submit(big)                 # needs more than the whole arena
        assert e.value.status == -2
        for bad in (job(2, p=3), job(3, l=0), job(4, kind=7), job(5, k=0),
                    bs.JobDesc(id=7, kind=bs.JOB_SKETCH, n=4096, m=8, p=4, l=2048,
                               sampling=bs.WITHOUT_REPLACEMENT, precision=bs.FP32, lda=8,
                               ldy=8),
                    bs.JobDesc(id=8, kind=bs.JOB_SKETCH, n=4096, m=8, p=4, l=64,
                               sampling=0, precision=5, lda=8, ldy=8),
                    bs.JobDesc(id=9, kind=bs.JOB_SKETCH, n=4096, m=8, p=4, l=64,
                               sampling=0, precision=0, lda=4, ldy=8)):
            with pytest.raises(bs.BsrhtError) as e:
                srv.submit(bad)
            assert e.value.status == -1
        assert srv.stats()["rejected"] == 8
        assert srv.stats()["submitted"] == 0


def test_backfill_admits_small_jobs_without_starving_the_large_one():
    small = job(0)
    large = job(1, n=1 << 16, m=512, l=256, k=64)
    b_small, b_large = bs.bsrht_job_bytes(small), bs.bsrht_job_bytes(large)
    assert b_large > 2 * b_small
    budget = b_large + b_small // 2      # the large job fits only when the arena is empty
    with bs.Server(fake_bytes=budget, workers=4, seconds_per_gb=5.0) as srv:
        srv.submit(job(100))              # a small job occupies part of the arena
        time.sleep(0.01)
        srv.submit(large)                 # cannot be admitted yet
        for i in range(3):
            srv.submit(job(200 + i, seed=7))
        srv.drain()
        res = {r.id: r for r in srv.poll(64)}
        st = srv.stats()
    assert len(res) == 5
    assert st["backfilled"] >= 1
    assert st["peak_arena_bytes"] <= budget
    # the large job was not starved: it started within the bypass bound after
    # the first small job finished, or as soon as the arena emptied
    first_done = res[100].t_done
    assert res[1].t_start >= first_done
    assert res[1].t_start - first_done < 0.1 + 3 * (res[100].t_done - res[100].t_start) + 0.05


def test_plan_cache_evicts_unused_plans_under_pressure():
    one = bs.bsrht_job_bytes(job(0))
    tables = bs.bsrht_plan_bytes(1 << 14, 4, 64)
    budget = one + tables // 2           # one job's workspace and 1.5 plans' tables
    with bs.Server(fake_bytes=budget, workers=1, seconds_per_gb=0.0) as srv:
        run_all(srv, [job(i, seed=i) for i in range(10)])   # ten different plans
        st = srv.stats()
    assert st["plan_misses"] == 10
    assert st["plan_evictions"] == 9
    assert st["peak_arena_bytes"] <= budget


def test_concurrent_submitters():
    with bs.Server(fake_bytes=1 << 30, workers=4, seconds_per_gb=0.1) as srv:
        def client(base):
            for i in range(50):
                srv.submit(job(base + i, seed=(base + i) % 5))
        ts = [threading.Thread(target=client, args=(1000 * t,)) for t in range(4)]
        for t in ts:
            t.start()
        got = []
        while len(got) < 200:
            got += srv.poll(64, timeout=1.0)
        for t in ts:
            t.join()
        ids = sorted(r.id for r in got)
        assert ids == sorted(1000 * t + i for t in range(4) for i in range(50))
        st = srv.stats()
        assert st["plan_misses"] == 5 and st["plan_hits"] == 195


def test_invalid_server_arguments():
    L = bs.lib()
    import ctypes
    h = ctypes.c_void_p()
    assert L.bsrht_server_create_fake(0, 2, 0.0, ctypes.byref(h)) == -1
    assert L.bsrht_server_create_fake(1 << 20, 0, 0.0, ctypes.byref(h)) == -1
    assert L.bsrht_server_create_fake(1 << 20, 65, 0.0, ctypes.byref(h)) == -1
    assert L.bsrht_server_create_fake(1 << 20, 2, -1.0, ctypes.byref(h)) == -1
    assert L.bsrht_server_create(None, 1 << 20, 2, ctypes.byref(h)) == -1
    assert L.bsrht_server_create(ctypes.c_void_p(4096 + 8), 1 << 20, 2, ctypes.byref(h)) == -1
    assert L.bsrht_server_create(ctypes.c_void_p(4096), 1 << 20, 0, ctypes.byref(h)) == -1


def test_submit_many_stops_at_the_first_rejected_job():
    with bs.Server(fake_bytes=1 << 30, workers=3, seconds_per_gb=0.1) as srv:
        assert srv.submit_many([job(i) for i in range(5)]) == 5
        with pytest.raises(bs.BsrhtError) as e:
            srv.submit_many([job(10), job(11), job(12, p=3), job(13)])
        assert e.value.status == -1
        srv.drain()
        res = srv.poll(64)
        assert sorted(r.id for r in res) == [0, 1, 2, 3, 4, 10, 11]
        st = srv.stats()
        assert st["submitted"] == 7 and st["rejected"] == 1 and st["completed"] == 7
        assert srv.submit_many([]) == 0


def test_nystrom_jobs_are_sized_and_validated():
    """A Nystrom job needs a square A (m == n); its arena bytes are the
    nystrom workspace plus the plan tables, and the scheduler runs it like
    the other kinds."""
    nys = job(0, n=1 << 12, m=1 << 12, p=4, l=64, k=16, kind=bs.JOB_NYSTROM)
    need = bs.bsrht_job_bytes(nys)
    assert need > 0
    bad = job(1, n=1 << 12, m=100, p=4, l=64, k=16, kind=bs.JOB_NYSTROM)
    assert bs.bsrht_job_bytes(bad) == 0
    bad_k = job(2, n=1 << 12, m=1 << 12, p=4, l=64, k=0, kind=bs.JOB_NYSTROM)
    assert bs.bsrht_job_bytes(bad_k) == 0
    jobs = [job(i, n=1 << 12, m=1 << 12, p=4, l=64, k=16, kind=bs.JOB_NYSTROM)
            for i in range(6)] + [job(10 + i) for i in range(6)]
    with bs.Server(fake_bytes=1 << 30, workers=3, seconds_per_gb=0.5) as srv:
        res = run_all(srv, jobs)
        assert all(r.status == 0 for r in res)
        held = {r.id: r.arena_bytes for r in res}
        assert held[0] == need      # the first Nystrom job built its plan
    with bs.Server(fake_bytes=1 << 30, workers=1) as srv:
        with pytest.raises(bs.BsrhtError):
            srv.submit(bad)
