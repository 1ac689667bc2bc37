#!/usr/bin/env python3
"""Benchmark of the block SRHT sketch Y = Omega A on one MI355X.

Workload (the large sketch case): A is 2^20 x 1024 float32, A = X diag(s) W^T
with X Gaussian / sqrt(n), W Haar, s_j = exp(-j/64), seed 0; Omega has
p = 16 blocks of r = 65536 rows and l = 512 samples.  A step is one sketch of
the whole matrix (every block's signs, Walsh-Hadamard transform, row sample,
output signs and the sum over blocks), with A resident in HBM.  Before the
warmup steps the bench runs --settle untimed sketches (default 100): after
the FP64 generation of A the GPU's clocks take ~20-30 ms of continuous load
to settle, and launches in that window run up to 30% slower.  The split-BF16
and right-side legs settle the same way.

Prints one JSON line: GB/s of A streamed, the dominant kernel's roofline
(achieved vs the 8 TB/s HBM peak, from HIP events around that kernel), and the
FP64 CPU oracle timed on a sample of the same workload; then the split-BF16
sketch, the randomized SVD and Nystrom at full size, and the serving workload
(Poisson arrivals of sketch + RSVD jobs).  Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The serving leg keeps up to 16 jobs in flight on 16 streams; HIP maps
# streams onto this many hardware queues (its default of 4 would serialise
# them).  Must be set before the HIP runtime starts.
os.environ["GPU_MAX_HW_QUEUES"] = "16"
SERVE_STREAMS = 16

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2210_11295_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(profile_name, src_files, bytes_per_launch_alg):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(path):
        return None
    try:
        doc = json.load(open(path))
    except (OSError, ValueError):
        return None
    if doc.get("source_sha256_16") != _src_hash(*src_files):
        return None
    return doc.get("hbm_bytes_per_launch")


def _cpu_facts():
    """CPU model, the cores this process may run on, and the BLAS threads."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        import threadpoolctl
        blas = [d.get("num_threads") for d in threadpoolctl.threadpool_info()
                if d.get("user_api") == "blas"]
    except Exception:  # noqa: BLE001 - informational only
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)),
            "blas_threads": blas}


def _rel_errors(Y, Y_ref):
    """Relative Frobenius error and largest entry error relative to max|Y_ref|."""
    Yh = Y.detach().cpu().double().numpy()
    D = Yh - Y_ref
    return {"rel_fro": float(np.linalg.norm(D) / np.linalg.norm(Y_ref)),
            "max_entry_rel": float(np.abs(D).max() / np.abs(Y_ref).max())}


def cpu_baseline(bs, A, cfg, Y_fp32, Y_bf16, blocks=8):
    """The cpu_baseline leg: the FP64 oracle on the host cores.

    Timing: the oracle's sketch (numpy FP64 FWHT) on one core, on a bounded
    sample (the first `blocks` row blocks of A as a plan with p = blocks and
    the same r, l and seed: the tables of block i depend only on (seed, i), so
    this is exactly the partial sum of the first terms of (2.4)); and on all
    cores (oracle.sketch.sketch_parallel: the same per-block terms on a
    thread per core, bitwise the sequential result) over the whole input.
    `value` is the all-core rate, as GB/s of FP32 A.

    Reference errors (FP64 oracle, same plan and FP32 input): the full-size
    FP32 and split-BF16 sketches of the benchmark; on A_sub = A[0:r] as a
    p = 1 plan (block 0 of the same tables) the two sketches again and the
    rank-k randomized SVD error against the oracle's."""
    import torch
    from oracle import lowrank, metrics, rng, sketch

    n, m, p, l, k, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["k"], cfg["seed"]
    r = n // p
    facts = _cpu_facts()
    workers = facts["affinity_cores"]
    Ah = A.cpu().numpy()

    blocks = min(blocks, p)
    op = rng.Plan(blocks * r, blocks, l, seed)
    t0 = time.perf_counter()
    Ys = sketch.sketch(op, Ah[:blocks * r])
    dt1 = time.perf_counter() - t0
    assert np.isfinite(Ys).all()
    gbs1 = blocks * r * m * 4 / dt1 / 1e9
    log(f"bench: oracle sketch, one core: {blocks} blocks in {dt1:.2f} s -> {gbs1:.4f} GB/s")

    t0 = time.perf_counter()
    Y_ref = sketch.sketch_parallel(rng.Plan(n, p, l, seed), Ah, workers=workers)
    dtn = time.perf_counter() - t0
    gbsn = n * m * 4 / dtn / 1e9
    log(f"bench: oracle sketch, {workers} threads: whole input in {dtn:.2f} s -> {gbsn:.4f} GB/s")

    errs = {"full_fp32": _rel_errors(Y_fp32, Y_ref)}
    if Y_bf16 is not None:
        errs["full_split_bf16"] = _rel_errors(Y_bf16, Y_ref)
    del Y_ref

    sub_op = rng.Plan(r, 1, l, seed)
    Asub = A[:r].contiguous()
    Ysub_ref = sketch.sketch(sub_op, Ah[:r])
    for name, prec in (("sub_fp32", bs.FP32), ("sub_split_bf16", bs.SPLIT_BF16)):
        Ysub = bs.bsrht_apply(bs.Plan(r, 1, l, seed, precision=prec, device=A.device), Asub)
        torch.cuda.synchronize()
        errs[name] = _rel_errors(Ysub, Ysub_ref)
    sub_plan = bs.Plan(r, 1, l, seed, device=A.device)
    U, S, V, info = bs.rsvd(sub_plan, Asub, k)
    torch.cuda.synchronize()
    Asub_h = Ah[:r].astype(np.float64)
    e_gpu = metrics.lowrank_fro_error(Asub_h, U.cpu().double().numpy(),
                                      S.cpu().double().numpy(), V.cpu().double().numpy())
    Uo, So, Vo = lowrank.rsvd(sub_op, Asub_h, k)
    e_or = metrics.lowrank_fro_error(Asub_h, Uo, So, Vo)
    errs["sub_rsvd"] = {"k": k, "l": l, "gpu_rel_fro_error": e_gpu, "oracle_rel_fro_error": e_or,
                        "ratio": e_gpu / e_or}
    log(f"bench: errors against the FP64 oracle: {json.dumps(errs)}")
    del Asub, Asub_h, Ah
    return {"value": round(gbsn, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"all cores: the whole {n} x {m} float32 input (p={p}, l={l}, seed "
                      f"{seed}), numpy FP64 FWHT, one thread per core over (block, column "
                      f"slice) terms summed in block order; {dtn:.2f} s",
            "one_core": {"value": round(gbs1, 4), "unit": "GB/s", "cores": 1,
                         "seconds": round(dt1, 2),
                         "sample": f"first {blocks} of {p} row blocks: {blocks * r} x {m} float32 "
                                   f"rows of A as a p={blocks} plan (same r, l, seed); "
                                   f"numpy FP64 FWHT, single thread"},
            **facts,
            "errors_vs_fp64_oracle": errs,
            "sub_workload": f"A_sub = A[0:{r}] (block 0) as a p=1 plan, l={l}, seed {seed}"}


def cpu_oracle_nystrom(bs, plan, cfg, A, X, s, trace_err):
    """cpu_baseline leg, Nystrom workload: the reference trace errors beside
    the GPU's (section 8d's three errors).

    oracle: Algorithm 2 in FP64 on the host for the exact A = X diag(s) X^T,
        through its structure: W = Omega A = (Omega X) diag(s) X^T with Omega X
        from the oracle's sketch, Y = W^T, B = Omega Y, then the oracle's
        steps 2-6 (oracle.lowrank.nystrom_from_sketch);
    hybrid: the GPU's FP32 sketches (W = Omega A and B = Omega W^T, the
        library's two sketch passes on the FP32 A) factored by those same
        FP64 host steps, which isolates the precision of the sketch.
    The errors are evaluated like the GPU's (trace_err: the eigenvalues of
    A - U diag(lam) U^T on span[X, U])."""
    import torch
    from oracle import lowrank, rng, sketch

    n, p, l, k, seed = cfg["n"], cfg["p"], cfg["l"], cfg["k"], cfg["seed"]
    workers = len(os.sched_getaffinity(0))
    dev = A.device
    t0 = time.perf_counter()
    op = rng.Plan(n, p, l, seed)
    Xh = X.cpu().numpy()
    sh = s.cpu().numpy()
    OX = sketch.sketch_parallel(op, Xh, workers=workers)           # Omega X (l x d)
    Yo = ((OX * sh[None, :]) @ Xh.T).T                              # Y = A Omega^T
    Bo = sketch.sketch_parallel(op, Yo, workers=workers)           # Omega Y
    Uo, lo, fbo = lowrank.nystrom_from_sketch(Yo, Bo, k, l)
    e_or = trace_err(torch.from_numpy(Uo).to(dev), torch.from_numpy(lo).to(dev))
    del Xh, OX, Yo, Bo, Uo
    t1 = time.perf_counter()
    W = bs.bsrht_apply(plan, A)
    Yg = W.t().contiguous()
    del W
    Bg = bs.bsrht_apply(plan, Yg)
    torch.cuda.synchronize()
    Uh, lh, fbh = lowrank.nystrom_from_sketch(Yg.cpu().double().numpy(),
                                              Bg.cpu().double().numpy(), k, l)
    del Yg, Bg
    e_hy = trace_err(torch.from_numpy(Uh).to(dev), torch.from_numpy(lh).to(dev))
    t2 = time.perf_counter()
    log(f"bench: nystrom reference errors: oracle {e_or:.3e} (fallback {fbo}, {t1 - t0:.1f} s), "
        f"hybrid {e_hy:.3e} (fallback {fbh}, {t2 - t1:.1f} s)")
    return {"oracle_trace_rel_error": e_or, "oracle_fallback": bool(fbo),
            "hybrid_trace_rel_error": e_hy, "hybrid_fallback": bool(fbh),
            "oracle_note": "FP64 oracle on the exact A = X diag(s) X^T (the FP32 rounding of A "
                           "is not seen by it); hybrid = GPU FP32 sketches, FP64 host factors"}


def _copy_calibration(A):
    """One plain device copy of A: reads and writes exactly A's bytes, the
    reference against which the HBM byte counters are scaled."""
    import torch
    log("bench: copy calibration")
    B = torch.empty_like(A)
    B.copy_(A)
    torch.cuda.synchronize()
    del B


def _kernel_stats(bs):
    """Median / p10 / p90 of the per-launch kernel times recorded since
    timing_enable, in microseconds."""
    us = np.array(bs.timing_samples(), dtype=np.float64) * 1e3
    if us.size == 0:
        return {}
    return {"kernel_median_us": round(float(np.median(us)), 2),
            "kernel_p10_us": round(float(np.percentile(us, 10)), 2),
            "kernel_p90_us": round(float(np.percentile(us, 90)), 2)}


def bench_stream_read(bs, A, reps=20, warmup=3):
    """Read-only reference over the same buffer: one pass of the library's
    plain read kernel (16-byte non-temporal loads) per repetition."""
    import torch
    out = torch.empty(bs.STREAM_BLOCKS, dtype=torch.float32, device=A.device)
    for _ in range(warmup):
        bs.stream_read(A, out)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_STREAM)
    for _ in range(reps):
        bs.stream_read(A, out)
    torch.cuda.synchronize()
    stats = _kernel_stats(bs)
    bs.timing_enable(bs.TIMING_OFF)
    gbs = A.numel() * 4 / (stats["kernel_median_us"] * 1e-6) / 1e9
    log(f"bench: read-only reference {gbs:.1f} GB/s (median of {reps})")
    return {"GBs": round(gbs, 2), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "stream_read_kernel", "reps": reps, **stats}


def bench_split_bf16(bs, A, cfg, steps, warmup, Y_fp32, settle=0):
    """The same sketch with the H_16 factor on BF16 matrix cores (A split
    into BF16 hi + lo, FP32 accumulation), on the same A and plan seed."""
    import torch
    n, m, p, l, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["seed"]
    plan = bs.Plan(n, p, l, seed, precision=bs.SPLIT_BF16, device=A.device)
    Y = torch.empty(l, m, dtype=torch.float32, device=A.device)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8,
                     device=A.device)
    stream = torch.cuda.current_stream()
    for _ in range(settle + warmup):
        bs.bsrht_apply(plan, A, Y, ws, stream)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_APPLY_BF16)
    t0 = time.perf_counter()
    for _ in range(steps):
        bs.bsrht_apply(plan, A, Y, ws, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = bs.timing_read()
    stats = _kernel_stats(bs)
    bs.timing_enable(bs.TIMING_OFF)
    kern_avg_ms = kern_ms / max(launches, 1)
    bytes_a = n * m * 4
    table_bytes = 4 * l + 4 * ((n + 31) // 32) + 4 * p * ((l + 31) // 32)
    alg_bytes = bytes_a + 4 * l * m + table_bytes
    achieved = alg_bytes / (kern_avg_ms * 1e-3) / 1e9
    diff = float((Y.double() - Y_fp32.double()).norm() / Y_fp32.double().norm())
    log(f"bench: split-bf16 {bytes_a * steps / elapsed / 1e9:.1f} GB/s whole call; kernel "
        f"{kern_avg_ms * 1e3:.1f} us -> {achieved:.1f} GB/s; rel diff vs fp32 {diff:.2e}")
    traffic = _traffic("traffic_fused_bf16_sketch_2p20x1024.json", ["apply_bf16.hip"],
                       alg_bytes)
    return {"value": round(bytes_a * steps / elapsed / 1e9, 2), "unit": "GB/s",
            "ms_per_step": round(elapsed / steps * 1e3, 4),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": traffic, "kernel": "fused_bf16_kernel<8, 64, false>",
                         "kernel_avg_us": round(kern_avg_ms * 1e3, 2), **stats,
                         "alg_bytes_per_launch": alg_bytes},
            "rel_diff_vs_fp32": diff}, Y


def bench_right(bs, A, cfg, steps, warmup, Y_col, settle=0):
    """The sketch applied from the right, Y = A^T Omega^T, on the transpose of
    the same input (1024 x 2^20 row-major: the orientation of Algorithm 1),
    with the same plan; compared with the column sketch of A."""
    import torch
    n, m, p, l, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["seed"]
    At = A.t().contiguous()
    plan = bs.Plan(n, p, l, seed, device=A.device)
    Y = torch.empty(m, l, dtype=torch.float32, device=A.device)
    ws = torch.empty(max(1, bs.bsrht_apply_right_workspace(plan, m)), dtype=torch.uint8,
                     device=A.device)
    stream = torch.cuda.current_stream()
    for _ in range(settle + warmup):
        bs.bsrht_apply_right(plan, At, Y, ws, stream)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_APPLY_RIGHT)
    t0 = time.perf_counter()
    for _ in range(steps):
        bs.bsrht_apply_right(plan, At, Y, ws, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = bs.timing_read()
    stats = _kernel_stats(bs)
    bs.timing_enable(bs.TIMING_OFF)
    kern_avg_ms = kern_ms / max(launches, 1)
    bytes_a = n * m * 4
    table_bytes = 4 * l + 4 * ((n + 31) // 32) + 4 * p * ((l + 31) // 32)
    alg_bytes = bytes_a + 4 * l * m + table_bytes
    achieved = alg_bytes / (kern_avg_ms * 1e-3) / 1e9
    diff = float((Y.double() - Y_col.double().t()).norm() / Y_col.double().norm())
    log(f"bench: right apply {bytes_a * steps / elapsed / 1e9:.1f} GB/s whole call; kernel "
        f"{kern_avg_ms * 1e3:.1f} us -> {achieved:.1f} GB/s; rel diff vs column sketch "
        f"{diff:.2e}")
    traffic = _traffic("traffic_right_fp32_sketch_1024x2p20.json", ["apply_right.hip"],
                       alg_bytes)
    del At
    return {"value": round(bytes_a * steps / elapsed / 1e9, 2), "unit": "GB/s",
            "ms_per_step": round(elapsed / steps * 1e3, 4),
            "workload": f"Y = A Omega^T, A {m} x {n} float32 row-major (the transpose of the "
                        f"column workload), p={p}, l={l}, seed {seed}",
            "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": traffic, "kernel": "right_fp32_kernel<8, false>",
                         "kernel_avg_us": round(kern_avg_ms * 1e3, 2), **stats,
                         "alg_bytes_per_launch": alg_bytes},
            "rel_diff_vs_column_sketch": diff}


def bench_dense(bs, A, cfg, steps, warmup, bsrht_ms):
    """The dense comparison sketches of section 4 on the same A and l: a
    Gaussian and a Rademacher G (l x n) generated into the workspace, then
    Y = G A on the FP32 matrix cores.  bsrht_ms: the block SRHT sketch's
    time per call on the same input."""
    import torch
    n, m, l, seed = cfg["n"], cfg["m"], cfg["l"], cfg["seed"]
    ws = torch.empty(max(1, bs.bsrht_dense_workspace(n, l, m)), dtype=torch.uint8,
                     device=A.device)
    Y = torch.empty(l, m, dtype=torch.float32, device=A.device)
    out = {}
    for name, kind in (("gaussian", bs.DENSE_GAUSSIAN), ("rademacher", bs.DENSE_RADEMACHER)):
        for _ in range(warmup):
            bs.bsrht_dense_sketch(kind, seed, l, A, Y, ws)
        torch.cuda.synchronize()
        bs.timing_enable(bs.TIMING_DENSE_GEMM)
        t0 = time.perf_counter()
        for _ in range(steps):
            bs.bsrht_dense_sketch(kind, seed, l, A, Y, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        gms, gl = bs.timing_read()
        bs.timing_enable(bs.TIMING_OFF)
        gemm_ms = gms / max(gl, 1)
        flops = 2.0 * l * m * n
        tf = flops / (gemm_ms * 1e-3) / 1e12
        log(f"bench: dense {name} sketch {dt * 1e3:.2f} ms per call, product {gemm_ms:.2f} ms "
            f"-> {tf:.1f} TFLOP/s; block SRHT {bsrht_ms:.3f} ms")
        out[name] = {"ms_per_call": round(dt * 1e3, 3), "product_ms": round(gemm_ms, 3),
                     "generate_ms": round(dt * 1e3 - gemm_ms, 3),
                     "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 157.3,
                                  "unit": "TFLOP/s", "frac": round(tf / 157.3, 4),
                                  "kernel": "gemm_big_kernel<float, float, double> split-K + "
                                            "reduce_partials_kernel",
                                  "alg_flops_per_launch": flops},
                     "bsrht_speedup": round(dt * 1e3 / bsrht_ms, 2)}
    del ws
    return out


def bench_partial(bs, steps=10, warmup=2, calibrate=False, settle=0):
    """The partial block SRHT (section 2: blocks padded with zeros to a power
    of two) on section 4.2's tall-skinny shape on one GPU: A 10^7 x 200 FP32
    (8 GB), p = 16 (r = 625000 rows, padded to 2^20), l = 2000.  l > 1024
    samples take two sample groups of workgroups (1024 samples each), each
    streaming A; the two groups of a tile run together on one XCD, so most of
    the second group's reads hit in cache (the HBM counters give the bytes)."""
    import torch
    import workloads
    n, m, p, l, seed = 10 ** 7, 200, 16, 2000, 0
    dev = torch.device("cuda:0")
    A = workloads.gaussian_cols(n, m, "inv_sq", seed, device=dev)
    plan = bs.Plan(n, p, l, seed, device=dev)
    Y = torch.empty(l, m, dtype=torch.float32, device=dev)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8, device=dev)
    for _ in range(settle + warmup):
        bs.bsrht_apply(plan, A, Y, ws)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_APPLY_FP32)
    t0 = time.perf_counter()
    for _ in range(steps):
        bs.bsrht_apply(plan, A, Y, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    kms, kl = bs.timing_read()
    stats = _kernel_stats(bs)
    bs.timing_enable(bs.TIMING_OFF)
    kern_ms = kms / max(kl, 1)
    groups = (l + 1023) // 1024
    # A, Y and the tables the kernel reads: R and the lane order (l int32
    # each), the D bits of the stored rows, the Dt bits
    alg = n * m * 4 + l * m * 4 + 8 * l + 4 * ((n + 31) // 32) + 4 * p * ((l + 31) // 32)
    achieved = alg / (kern_ms * 1e-3) / 1e9
    log(f"bench: partial block SRHT n=1e7: {dt * 1e3:.3f} ms per call, kernel {kern_ms:.3f} ms "
        f"-> {achieved:.1f} GB/s ({groups} sample groups)")
    if calibrate:
        _copy_calibration(A)
    del A, ws
    torch.cuda.empty_cache()
    traffic = _traffic("traffic_partial_fp32_sketch_1e7x200_l2000.json", ["apply_fp32.hip"], alg)
    return {"workload": f"A {n} x {m} float32, p={p} (r={n // p} padded to {plan.rp}), l={l}, "
                        f"seed {seed}", "ms_per_call": round(dt * 1e3, 3),
            "GBs_of_A": round(n * m * 4 / dt / 1e9, 1), "sample_groups": groups,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": traffic,
                         "kernel": "fused_fp32_kernel<16, 16, true>",
                         "kernel_avg_us": round(kern_ms * 1e3, 2), **stats,
                         "alg_bytes_per_launch": alg}}


def bench_nystrom_sketch(bs, steps=10, warmup=2, settle=20):
    """The two sketches of Algorithm 2 on the 65536 x 65536 SPD input
    (p = 64, r = 1024, l = 1024: the 16-wave kernels): W = Omega A over the
    16 GiB A, then B = Omega Y over Y = W^T (65536 x 1024), in both
    precisions.  Per-launch kernel times of each pass; the roofline takes
    the algorithmic bytes of both passes (A and Y read once, W and B
    written, tables) over the summed kernel time."""
    import torch
    import workloads
    c = workloads.CONFIGS["c5_nystrom"]
    n, l, p = c["n"], c["l"], c["p"]
    dev = torch.device("cuda:0")
    log(f"bench: nystrom sketches, generating SPD {n}x{n}")
    A = workloads.spd(n, c["d"], c["spectrum"], c["seed"], device=dev)
    tables = 8 * l + 4 * ((n + 31) // 32) + 4 * p * ((l + 31) // 32)
    alg = (n * n * 4 + l * n * 4 + tables) + (n * l * 4 + l * l * 4 + tables)
    out = {"workload": f"A {n} x {n} float32 (s_j = j^-3), p={p}, l={l}; "
                       f"W = Omega A, then B = Omega W^T", "alg_bytes_both_passes": alg}
    for name, prec, hook, kern in (
            ("fp32", bs.FP32, bs.TIMING_APPLY_FP32, "fused_fp32_kernel<16, 16>"),
            ("split_bf16", bs.SPLIT_BF16, bs.TIMING_APPLY_BF16, "fused_bf16_kernel<16, 16>")):
        plan = bs.Plan(n, p, l, c["seed"], precision=prec, device=dev)
        W = torch.empty(l, n, dtype=torch.float32, device=dev)
        Y = torch.empty(n, l, dtype=torch.float32, device=dev)
        B = torch.empty(l, l, dtype=torch.float32, device=dev)
        ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, n),
                             bs.bsrht_apply_workspace(plan, l)), dtype=torch.uint8, device=dev)
        for _ in range(settle):
            bs.bsrht_apply(plan, A, W, ws)
        for _ in range(warmup):
            bs.bsrht_apply(plan, A, W, ws)
            Y.copy_(W.t())
            bs.bsrht_apply(plan, Y, B, ws)
        torch.cuda.synchronize()
        bs.timing_enable(hook)
        for _ in range(steps):
            bs.bsrht_apply(plan, A, W, ws)
            Y.copy_(W.t())
            bs.bsrht_apply(plan, Y, B, ws)
        torch.cuda.synchronize()
        t = np.array(bs.timing_samples(), dtype=np.float64) * 1e3
        bs.timing_enable(bs.TIMING_OFF)
        ta, ty = t[0::2], t[1::2]
        both = float(ta.mean() + ty.mean())
        achieved = alg / (both * 1e-6) / 1e9
        out[name] = {"pass_A_us": round(float(ta.mean()), 1),
                     "pass_A_median_us": round(float(np.median(ta)), 1),
                     "pass_Y_us": round(float(ty.mean()), 1),
                     "both_passes_ms": round(both / 1e3, 4),
                     "A_GBs": round(n * n * 4 / (ta.mean() * 1e-6) / 1e9, 1),
                     "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": kern}}
        log(f"bench: nystrom sketches {name}: A pass {ta.mean():.1f} us, Y pass "
            f"{ty.mean():.1f} us -> {achieved:.1f} GB/s")
        del W, Y, B, ws
    del A
    torch.cuda.empty_cache()
    return out


def launch_sequence(bs, A, plan, count=60, gap_s=0.002):
    """Diagnostic: per-launch durations of the fused sketch kernel in launch
    order, for `count` launches back to back, then with `gap_s` of idle time
    between launches, then back to back again (GPU clock and power-state
    transients show up as runs of slower launches)."""
    import torch
    Y = torch.empty(plan.l, A.shape[1], device=A.device)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, A.shape[1])), dtype=torch.uint8,
                     device=A.device)
    for _ in range(5):
        bs.bsrht_apply(plan, A, Y, ws)
    torch.cuda.synchronize()
    out = {}
    for mode in ("back_to_back", "with_gaps", "back_to_back_again"):
        bs.timing_enable(bs.TIMING_APPLY_FP32)
        for _ in range(count):
            bs.bsrht_apply(plan, A, Y, ws)
            if mode == "with_gaps":
                torch.cuda.synchronize()
                time.sleep(gap_s)
        torch.cuda.synchronize()
        t = np.array(bs.timing_samples(), dtype=np.float64) * 1e3
        bs.timing_enable(bs.TIMING_OFF)
        out[mode] = {"mean_us": round(float(t.mean()), 1), "median_us": round(float(np.median(t)), 1),
                     "min_us": round(float(t.min()), 1), "max_us": round(float(t.max()), 1),
                     "launch_us": [round(float(x), 1) for x in t]}
        log(f"bench: {mode}: mean {t.mean():.1f} us, median {np.median(t):.1f}, "
            f"min {t.min():.1f}, max {t.max():.1f}")
    return out


def _fro_error(A, U, S, V, chunk=1 << 16):
    """||A - U diag(S) V^T||_F / ||A||_F in FP64 on the device (measurement)."""
    import torch
    SVt = (S.double()[:, None] * V.double().T)
    num = 0.0
    den = 0.0
    for r0 in range(0, A.shape[0], chunk):
        Ab = A[r0:r0 + chunk].double()
        E = Ab - U[r0:r0 + chunk].double() @ SVt
        num += float((E * E).sum())
        den += float((Ab * Ab).sum())
    return (num / den) ** 0.5


def bench_rsvd(bs, A, plan, cfg, reps):
    """Algorithm 1 at full size: rank k, l = 512, FP64 Cholesky-QR2 on the GPU."""
    import torch
    n, m, k = cfg["n"], cfg["m"], cfg["k"]
    ws = torch.empty(max(1, bs.rsvd_workspace(plan, m, k)), dtype=torch.uint8, device=A.device)
    log(f"bench: rsvd rank {k} (workspace {ws.numel() / 2**30:.2f} GiB)")
    U, S, V, info = bs.rsvd(plan, A, k, ws)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_GEMM_AQ)
    t0 = time.perf_counter()
    for _ in range(reps):
        U, S, V, info = bs.rsvd(plan, A, k, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    gms, gl = bs.timing_read()
    bs.timing_enable(bs.TIMING_OFF)
    lq = min(cfg["l"], m)
    gemm_ms = gms / max(gl, 1)
    err = _fro_error(A, U, S, V)
    # Z = A Q runs on the BF16 matrix cores with both operands split (six
    # products for an FP32 plan, three for a split-BF16 plan) when A's rows
    # are 16-byte aligned, as here
    products = 3 if plan.precision == bs.SPLIT_BF16 else 6
    alg = 2.0 * n * m * lq
    return {"ms": round(dt * 1e3, 2), "k": k, "l": cfg["l"],
            "precision": "split_bf16" if plan.precision == bs.SPLIT_BF16 else "fp32",
            "gemm_AQ_ms": round(gemm_ms, 3),
            "gemm_AQ": {"form": f"split-BF16 MFMA, {products} products",
                        "alg_TFLOPs": round(alg / (gemm_ms * 1e-3) / 1e12, 2),
                        "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": 2500.0,
                                     "achieved": round(products * alg / (gemm_ms * 1e-3) / 1e12,
                                                       1),
                                     "frac": round(products * alg / (gemm_ms * 1e-3) / 2.5e15,
                                                   4)}},
            "rel_fro_error": err, "info": int(info.item())}


def bench_single_view(bs, A, cfg, reps):
    """Algorithm 3 (single-view RSVD) at full size on the same A: rank k,
    Omega and Gamma with l = 512 rows, Phi and Psi with s = 2l = 1024 rows
    (Gamma, Phi: p = 16 over the 2^20 rows; Omega, Psi: p = 1 over the 1024
    columns, without replacement); A is read three times."""
    import torch
    n, m, p, l, k, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["k"], cfg["seed"]
    s = 2 * l
    dev = A.device
    # Omega and Psi sample the 1024 columns without replacement (a repeated
    # index of a p = 1 plan gives collinear sketch rows); Gamma and Phi draw
    # 512 and 1024 of 65536 per block with replacement.
    wor = bs.WITHOUT_REPLACEMENT
    plans = [bs.Plan(m, 1, l, seed + 1, wor, device=dev), bs.Plan(n, p, l, seed + 2, device=dev),
             bs.Plan(n, p, s, seed + 3, device=dev), bs.Plan(m, 1, s, seed + 4, wor, device=dev)]
    ws = torch.empty(max(1, bs.rsvd_single_view_workspace(*plans, k)), dtype=torch.uint8,
                     device=dev)
    log(f"bench: single-view rsvd rank {k} (workspace {ws.numel() / 2**30:.2f} GiB)")
    U, S, V, info = bs.rsvd_single_view(*plans, A, k, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        U, S, V, info = bs.rsvd_single_view(*plans, A, k, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    err = _fro_error(A, U, S, V)
    return {"ms": round(dt * 1e3, 2), "k": k, "l": l, "s": s, "passes_over_A": 3,
            "rel_fro_error": err, "info": int(info.item())}


def bench_serving(bs, njobs, streams, rate=200.0, arena_gib=32, out_gib=96):
    """Serving workload: Poisson arrivals at `rate` jobs/s of sketch + RSVD
    jobs with seeded random shapes (n = 2^a, a in 14..20; m log-uniform in
    [64, 2048]; p in {1, 4, 16, 64}; k in 16..256; l = 2k + 32).

    Payloads: A = X diag(j^-1.5) with Gaussian X.  One seeded pool
    P = X diag(j^-1.5) of 2^20 x 2048 FP32 is generated before the clock
    starts, and job i reads the n x m window of P at a seeded random row
    offset (leading dimension 2048), so preparing a payload costs neither GPU
    time nor client time and the latency measures the server.  Each job gets
    its own output tensors at submission.  Latency runs from the scheduled
    arrival to the server observing the job's completion event; a job is
    submitted late only when the outputs of unfinished jobs would exceed
    `out_gib` GiB (reported as max_submit_lag_ms)."""
    import numpy as np
    import torch
    import workloads

    dev = torch.device("cuda:0")
    jobs = workloads.serving_jobs(njobs, rate, seed=0)
    rows, cols = 1 << 20, 2048
    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    pool = torch.randn(rows, cols, generator=g, device=dev)
    pool *= torch.arange(1, cols + 1, device=dev, dtype=torch.float32) ** -1.5
    offs = np.random.default_rng(1).integers(0, rows, size=njobs)
    arena = torch.empty(arena_gib << 30, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"bench: serving {njobs} jobs at {rate:.0f}/s on {streams} stream slots, "
        f"arena {arena_gib} GiB, payloads from a {rows} x {cols} pool")
    lat, done_at = {}, {}
    live = {}          # submitted, not finished: id -> (output tensors, bytes)
    a_bytes = 0
    out_bytes = 0
    lag = 0.0

    import resource
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    with bs.Server(arena=arena, workers=streams) as srv:
        def collect(res):
            nonlocal out_bytes
            for r in res:
                if r.status != 0:
                    raise RuntimeError(f"serving job {r.id} failed with status {r.status}")
                lat[r.id] = r.t_done - (t0 + jobs[r.id]["arrival"])
                done_at[r.id] = r.t_done
                out_bytes -= live.pop(r.id)[1]

        t0 = srv.clock() + 0.05
        for js in jobs:
            n, m, k = js["n"], js["m"], js["k"]
            nb = 4 * (n * k + m * k) + 8 * k + 4
            while out_bytes + nb > (out_gib << 30) and live:
                collect(srv.poll(256, timeout=5e-4))
            while srv.clock() < t0 + js["arrival"]:
                collect(srv.poll(256, timeout=min(5e-4, max(t0 + js["arrival"] - srv.clock(),
                                                            5e-5))))
            off = int(offs[js["id"]]) % (rows - n + 1)
            A = pool[off:off + n, :m]
            U = torch.empty(n, k, device=dev)
            S = torch.empty(k, dtype=torch.float64, device=dev)
            V = torch.empty(m, k, device=dev)
            info = torch.empty(1, dtype=torch.int32, device=dev)
            lag = max(lag, srv.clock() - (t0 + js["arrival"]))
            live[js["id"]] = ((U, S, V, info), nb)
            out_bytes += nb
            srv.submit(bs.rsvd_job(js["id"], (n, js["p"], js["l"], 0, bs.WITH_REPLACEMENT,
                                              bs.FP32), A, k, U, S, V, info))
            a_bytes += n * m * 4
            collect(srv.poll(256))
            if js["id"] % 1000 == 999:
                log(f"bench: serving {js['id'] + 1} submitted, {len(lat)} done, "
                    f"{out_bytes / 2 ** 30:.1f} GiB of outputs live")
        srv.drain()
        collect(srv.poll(njobs))
        st = srv.stats()
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    del pool, arena
    torch.cuda.empty_cache()
    cpu_s = (ru1.ru_utime - ru0.ru_utime) + (ru1.ru_stime - ru0.ru_stime)
    L = np.array([lat[i] for i in range(njobs)]) * 1e3
    span = max(done_at.values()) - t0
    out = {"jobs": njobs, "offered_jobs_per_s": rate, "stream_slots": streams,
           "p50_ms": round(float(np.percentile(L, 50)), 3),
           "p99_ms": round(float(np.percentile(L, 99)), 3),
           "max_ms": round(float(L.max()), 3),
           "jobs_per_s": round(njobs / span, 2), "GBs_of_A": round(a_bytes / span / 1e9, 2),
           "max_submit_lag_ms": round(lag * 1e3, 3),
           "host_cpu_s_per_wall_s": round(cpu_s / span, 3),
           "peak_running": st["peak_running"], "peak_arena_GiB": round(
               st["peak_arena_bytes"] / 2 ** 30, 3),
           "plan_hits": st["plan_hits"], "plan_misses": st["plan_misses"],
           "plan_evictions": st["plan_evictions"], "backfilled": st["backfilled"],
           "rejected": st["rejected"],
           "payloads": "n x m windows (seeded row offsets) of one 2^20 x 2048 pool "
                       "X diag(j^-1.5), X Gaussian, generated before the clock starts"}
    log(f"bench: serving p50 {out['p50_ms']} ms p99 {out['p99_ms']} ms, "
        f"{out['jobs_per_s']} jobs/s, {out['GBs_of_A']} GB/s of A")
    return out


def bench_nystrom(bs, reps, with_oracle=False):
    """Algorithm 2 on the 65536 x 65536 SPD matrix (s_j = j^-3, p = 64, l = 1024,
    rank 512), FP64 factorisations on the GPU.  with_oracle: also the
    cpu_baseline leg's reference errors (cpu_oracle_nystrom)."""
    import torch
    import workloads
    c = workloads.CONFIGS["c5_nystrom"]
    n, l, k, p = c["n"], c["l"], c["k"], c["p"]
    dev = torch.device("cuda:0")
    log(f"bench: nystrom, generating SPD {n}x{n}")
    A, X, s = workloads.spd(n, c["d"], c["spectrum"], c["seed"], device=dev, return_factors=True)
    plan = bs.Plan(n, p, l, c["seed"], device=dev)
    ws = torch.empty(max(1, bs.nystrom_workspace(plan, k)), dtype=torch.uint8, device=dev)
    U, lam, info = bs.nystrom(plan, A, k, ws)
    torch.cuda.synchronize()
    bs.timing_enable(bs.TIMING_APPLY_FP32)
    t0 = time.perf_counter()
    for _ in range(reps):
        U, lam, info = bs.nystrom(plan, A, k, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    kms, kl = bs.timing_read()
    bs.timing_enable(bs.TIMING_OFF)
    # the sketch of A alone (16 GiB) in both precisions: GB/s of A
    apply = {}
    for name, prec, hook in (("fp32", bs.FP32, bs.TIMING_APPLY_FP32),
                             ("split_bf16", bs.SPLIT_BF16, bs.TIMING_APPLY_BF16)):
        pl = bs.Plan(n, p, l, c["seed"], precision=prec, device=dev)
        W = torch.empty(l, n, dtype=torch.float32, device=dev)
        aws = torch.empty(max(1, bs.bsrht_apply_workspace(pl, n)), dtype=torch.uint8, device=dev)
        bs.bsrht_apply(pl, A, W, aws)
        torch.cuda.synchronize()
        bs.timing_enable(hook)
        for _ in range(3):
            bs.bsrht_apply(pl, A, W, aws)
        torch.cuda.synchronize()
        ams, al = bs.timing_read()
        bs.timing_enable(bs.TIMING_OFF)
        apply[f"apply_{name}_GBs"] = round(n * n * 4 / (ams / al * 1e-3) / 1e9, 1)
        del W, aws
    def trace_err(U, lam):
        # A - U diag(lam) U^T lies in span[X, U]: eigenvalues of its compression
        B, _ = torch.linalg.qr(torch.cat([X, U.double()], dim=1))
        XtB = X.T @ B
        UtB = U.double().T @ B
        E = (XtB.T * s[None, :]) @ XtB - (UtB.T * lam[None, :]) @ UtB
        ev = torch.linalg.eigvalsh(0.5 * (E + E.T))
        return float(ev.abs().sum() / s.sum())

    err = trace_err(U, lam)
    opt = float(s[k:].sum() / s.sum())
    # the shifted variant (A + nu I, nu subtracted) on the same plan and A
    Us, lams, infos = bs.nystrom_shifted(plan, A, k, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Us, lams, infos = bs.nystrom_shifted(plan, A, k, ws)
    torch.cuda.synchronize()
    dts = (time.perf_counter() - t0) / reps
    shifted = {"ms": round(dts * 1e3, 2), "trace_rel_error": trace_err(Us, lams),
               "info": int(infos.item())}
    log(f"bench: nystrom {dt * 1e3:.1f} ms err {err:.3e} (info {int(info.item())}); shifted "
        f"{dts * 1e3:.1f} ms err {shifted['trace_rel_error']:.3e} (info {shifted['info']})")
    res = {"ms": round(dt * 1e3, 2), "n": n, "l": l, "k": k, "p": p,
           "sketch_kernel_ms_per_call": round(kms / max(reps, 1), 3), **apply,
           "trace_rel_error": err, "optimal_trace_rel_error": opt,
           "info": int(info.item()), "shifted": shifted}
    if with_oracle:
        del Us, U, ws
        torch.cuda.empty_cache()
        res.update(cpu_oracle_nystrom(bs, plan, c, A, X, s, trace_err))
    return res


def bench_serving_small(bs, njobs=3000, rate=None, streams=SERVE_STREAMS, seed=1):
    """Small FP32 sketch jobs (n = 2^a, a in 12..16; m log-uniform in
    [16, 512]; p in {1, 4, 16}; l in {64, 128, 256, 512}: 60 plans, which the
    server's cache keeps), submitted as one burst (or at
    Poisson arrivals of `rate` jobs/s), run once with the server's batched
    launches of small jobs and once with every job alone on a slot.  At
    offered rates the slots keep up with (tens of thousands of jobs/s) no
    batch ever forms; a backlog is where fusion acts, so the default is a
    burst.  Payloads are slices of a few device matrices prepared beforehand
    (inputs are read-only; each job has its own output).  Reports jobs/s
    (jobs over first arrival to last completion) and p50/p99 latency from the
    scheduled arrival."""
    import torch
    dev = torch.device("cuda:0")
    rs = np.random.default_rng(seed)
    t = np.cumsum(rs.exponential(1.0 / rate, size=njobs)) if rate else np.zeros(njobs)
    pool = [torch.randn(1 << 16, 512, device=dev) for _ in range(4)]
    jobs = []
    for i in range(njobs):
        n = 1 << int(rs.integers(12, 17))
        m = int(round(math.exp(rs.uniform(math.log(16), math.log(512)))))
        p = int(rs.choice([1, 4, 16]))
        l = min(int(rs.choice([64, 128, 256, 512])), n)
        A = pool[i % len(pool)][:n, :m]
        Y = torch.empty(l, m, device=dev)
        desc = bs.sketch_job(i, (n, p, l, 0, bs.WITH_REPLACEMENT, bs.FP32), A, Y)
        jobs.append((i, float(t[i]), desc, A, Y))
    torch.cuda.synchronize()
    arena = torch.empty(8 << 30, dtype=torch.uint8, device=dev)
    out = {"jobs": njobs, "offered_jobs_per_s": rate if rate else "burst",
           "stream_slots": streams}
    for mode in ("batched", "alone"):
        lat = {}
        with bs.Server(arena=arena, workers=streams) as srv:
            srv.set_batching(mode == "batched")
            t0 = srv.clock() + 0.02
            if rate:
                for (i, arr, desc, A, Y) in jobs:
                    while srv.clock() < t0 + arr:
                        for r in srv.poll(256):
                            lat[r.id] = r.t_done - (t0 + jobs[r.id][1])
                    srv.submit(desc)
            else:
                while srv.clock() < t0:
                    pass
                srv.submit_many([js[2] for js in jobs])
            srv.drain()
            for r in srv.poll(njobs):
                lat[r.id] = r.t_done - (t0 + jobs[r.id][1])
            st = srv.stats()
        L = np.array([lat[i] for i in range(njobs)]) * 1e3
        span = max(lat[i] + jobs[i][1] for i in range(njobs)) - jobs[0][1]
        out[mode] = {"jobs_per_s": round(njobs / span, 1),
                     "p50_ms": round(float(np.percentile(L, 50)), 3),
                     "p99_ms": round(float(np.percentile(L, 99)), 3),
                     "batches": st["batches"], "batched_jobs": st["batched_jobs"]}
        log(f"bench: small sketch serving ({mode}): {out[mode]}")
    del arena, pool
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle", type=int, default=100,
                    help="untimed sketch launches before the warmup steps (GPU clock settling)")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of A (HBM counter calibration)")
    ap.add_argument("--skip-lowrank", action="store_true",
                    help="skip the randomized SVD and Nystrom measurements")
    ap.add_argument("--lowrank-reps", type=int, default=3)
    ap.add_argument("--serve-jobs", type=int, default=10000,
                    help="jobs of the serving workload (0 skips it)")
    ap.add_argument("--serve-streams", type=int, default=SERVE_STREAMS)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--only", choices=["all", "sketch", "bf16", "right", "dense", "partial",
                                       "rsvd", "single_view", "nystrom", "serve",
                                       "serve_small", "launch_sequence", "nystrom_sketch"],
                    default="all",
                    help="profiling aid: run one part ('bf16', 'right', 'rsvd', 'nystrom' and "
                         "'serve' print only that part's JSON object)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sketch would shard by blocks with one l x m reduction)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2210_11295_amd as bs
    import workloads

    if args.only == "serve":
        print(json.dumps({"serving": bench_serving(bs, args.serve_jobs, args.serve_streams,
                                                   rate=args.serve_rate)}), flush=True)
        return
    if args.only == "serve_small":
        print(json.dumps({"serving_small_sketch": bench_serving_small(bs)}), flush=True)
        return
    if args.only == "nystrom_sketch":
        print(json.dumps({"nystrom_sketch": bench_nystrom_sketch(
            bs, steps=args.steps, warmup=args.warmup, settle=args.settle // 5)}), flush=True)
        return
    if args.only == "nystrom":
        print(json.dumps({"nystrom": bench_nystrom(bs, args.lowrank_reps,
                                                   with_oracle=not args.skip_cpu_baseline)}),
              flush=True)
        return
    if args.only == "partial":
        print(json.dumps({"partial_sketch": bench_partial(bs, calibrate=args.copy_calibration,
                                                          settle=args.settle // 5)}),
              flush=True)
        return
    cfg = dict(workloads.CONFIGS["c2_fp32_apply"])
    n, m, p, l, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["seed"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: generating A {n}x{m} float32 on {torch.cuda.get_device_name(dev)}")
    A = workloads.lowrank_tall(n, m, cfg["spectrum"], seed, device=dev)
    torch.cuda.synchronize()
    plan = bs.Plan(n, p, l, seed, device=dev)
    if args.only == "rsvd":
        print(json.dumps({"rsvd": bench_rsvd(bs, A, plan, cfg, args.lowrank_reps),
                          "rsvd_split_bf16": bench_rsvd(
                              bs, A, bs.Plan(n, p, l, seed, precision=bs.SPLIT_BF16, device=dev),
                              cfg, args.lowrank_reps)}), flush=True)
        return
    if args.only == "launch_sequence":
        print(json.dumps({"launch_sequence": launch_sequence(bs, A, plan)}), flush=True)
        return
    if args.only == "single_view":
        print(json.dumps({"rsvd_single_view": bench_single_view(bs, A, cfg, args.lowrank_reps)}),
              flush=True)
        return
    if args.only == "bf16":
        Yf = bs.bsrht_apply(plan, A)
        out_b, _ = bench_split_bf16(bs, A, cfg, args.steps, args.warmup, Yf,
                                   settle=args.settle)
        if args.copy_calibration:
            _copy_calibration(A)
        print(json.dumps({"split_bf16": out_b}), flush=True)
        return
    if args.only == "dense":
        bs.bsrht_apply(plan, A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            bs.bsrht_apply(plan, A)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t0) / 5 * 1e3
        print(json.dumps({"dense_sketch": bench_dense(bs, A, cfg, 5, 1, bms)}), flush=True)
        return
    if args.only == "right":
        Yf = bs.bsrht_apply(plan, A)
        out_r = bench_right(bs, A, cfg, args.steps, args.warmup, Yf, settle=args.settle)
        if args.copy_calibration:
            _copy_calibration(A)
        print(json.dumps({"right_apply": out_r}), flush=True)
        return
    Y = torch.empty(l, m, dtype=torch.float32, device=dev)
    Y_bf16 = None
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    # Settle: the GPU's clocks take ~20-30 ms of continuous sketching to
    # reach their steady state after the FP64 input generation (launches
    # right after it run up to 20% slower); these untimed launches come
    # before the warmup steps so that the timed steps measure the steady
    # state.
    log(f"bench: settle {args.settle}, warmup {args.warmup}")
    for _ in range(args.settle):
        bs.bsrht_apply(plan, A, Y, ws)
    for _ in range(args.warmup):
        bs.bsrht_apply(plan, A, Y, ws)
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    bs.timing_enable(bs.TIMING_APPLY_FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bs.bsrht_apply(plan, A, Y, ws, stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms, launches = bs.timing_read()
    stats = _kernel_stats(bs)
    bs.timing_enable(bs.TIMING_OFF)
    elapsed = t1 - t0
    bytes_a = n * m * 4
    value = bytes_a * args.steps / elapsed / 1e9
    kern_avg_ms = kern_ms / max(launches, 1)
    table_bytes = 4 * l + 4 * ((n + 31) // 32) + 4 * p * ((l + 31) // 32)
    alg_bytes = bytes_a + 4 * l * m + table_bytes
    achieved = alg_bytes / (kern_avg_ms * 1e-3) / 1e9
    log(f"bench: {value:.1f} GB/s whole call; fused kernel {kern_avg_ms * 1e3:.1f} us avg over "
        f"{launches} launches -> {achieved:.1f} GB/s")

    if args.copy_calibration:
        _copy_calibration(A)

    traffic = _traffic("traffic_fused_fp32_sketch_2p20x1024.json", ["apply_fp32.hip"], alg_bytes)
    stream_ref = bench_stream_read(bs, A)
    out = {
        "metric": "block-SRHT sketch GB/s of A (FP32 fused apply)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": args.settle,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; A = X diag(exp(-j/64)) W^T, X Gaussian, W Haar)",
        "config": {"workload": "block SRHT sketch, A 2^20 x 1024 float32, p=16 (r=65536), "
                               "l=512, seed 0", "n": n, "m": m, "p": p, "l": l,
                   "parallelism": "single GPU"},
        "frac_hbm_peak": round(value / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "fused_fp32_kernel<8, 64>",
                     "kernel_avg_us": round(kern_avg_ms * 1e3, 2), **stats,
                     "alg_bytes_per_launch": alg_bytes,
                     "frac_of_stream_read": round(achieved / stream_ref["GBs"], 4)},
        "stream_read": stream_ref,
    }
    if args.only == "sketch":
        args.skip_lowrank = True
    else:
        out["split_bf16"], Y_bf16 = bench_split_bf16(bs, A, cfg, args.steps, args.warmup, Y,
                                                     settle=args.settle)
        out["right_apply"] = bench_right(bs, A, cfg, args.steps, args.warmup, Y,
                                         settle=args.settle)
        out["dense_sketch"] = bench_dense(bs, A, cfg, 5, 1, elapsed / args.steps * 1e3)
    if not args.skip_lowrank:
        out["rsvd"] = bench_rsvd(bs, A, plan, cfg, args.lowrank_reps)
        out["rsvd_split_bf16"] = bench_rsvd(
            bs, A, bs.Plan(n, p, l, seed, precision=bs.SPLIT_BF16, device=dev), cfg,
            args.lowrank_reps)
        out["rsvd_single_view"] = bench_single_view(bs, A, cfg, args.lowrank_reps)
    if not args.skip_cpu_baseline:
        log("bench: the CPU oracle (timing and reference errors)")
        out["cpu_baseline"] = cpu_baseline(bs, A, cfg, Y, Y_bf16)
    if not args.skip_lowrank:
        del A, Y, ws
        torch.cuda.empty_cache()
        out["nystrom"] = bench_nystrom(bs, args.lowrank_reps,
                                       with_oracle=not args.skip_cpu_baseline)
        torch.cuda.empty_cache()
        out["partial_sketch"] = bench_partial(bs, settle=args.settle // 5)
    if args.serve_jobs > 0 and args.only == "all":
        out["serving"] = bench_serving(bs, args.serve_jobs, args.serve_streams,
                                       rate=args.serve_rate)
        out["serving_small_sketch"] = bench_serving_small(bs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
