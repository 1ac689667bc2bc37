#!/usr/bin/env python3
"""Benchmark of the block SRHT sketch Y = Omega A on one MI355X.

Workload (the large sketch case): A is 2^20 x 1024 float32, A = X diag(s) W^T
with X Gaussian / sqrt(n), W Haar, s_j = exp(-j/64), seed 0; Omega has
p = 16 blocks of r = 65536 rows and l = 512 samples.  A step is one sketch of
the whole matrix (every block's signs, Walsh-Hadamard transform, row sample,
output signs and the sum over blocks), with A resident in HBM.

Prints one JSON line: GB/s of A streamed, the dominant kernel's roofline
(achieved vs the 8 TB/s HBM peak, from HIP events around that kernel), and the
FP64 CPU oracle timed on a sample of the same workload.  Progress goes to
stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

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


def cpu_baseline(A, cfg):
    """The FP64 oracle sketch timed on host cores: the first block of A
    (2^16 rows x 1024 columns) as a p = 1 plan with the same r, l, seed."""
    import numpy as np
    from oracle import rng, sketch

    r = cfg["n"] // cfg["p"]
    sample = A[:r].cpu().numpy()
    op = rng.Plan(r, 1, cfg["l"], cfg["seed"])
    t0 = time.perf_counter()
    Y = sketch.sketch(op, sample)
    dt = time.perf_counter() - t0
    assert np.isfinite(Y).all()
    gbs = sample.size * 4 / dt / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first block: {r} x {cfg['m']} float32 rows of A as a p=1 plan "
                      f"(l={cfg['l']}); numpy FP64 FWHT, single thread; {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of A (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the sketch would shard by blocks with one l x m reduction)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2210_11295_amd as bs
    import workloads

    cfg = dict(workloads.CONFIGS["c2_fp32_apply"])
    n, m, p, l, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["seed"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: generating A {n}x{m} float32 on {torch.cuda.get_device_name(dev)}")
    A = workloads.lowrank_tall(n, m, cfg["spectrum"], seed, device=dev)
    torch.cuda.synchronize()
    plan = bs.Plan(n, p, l, seed, device=dev)
    Y = torch.empty(l, m, dtype=torch.float32, device=dev)
    ws = torch.empty(max(1, bs.bsrht_apply_workspace(plan, m)), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    log(f"bench: warmup {args.warmup}")
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
        # one plain copy of A: reads and writes exactly n*m*4 bytes, the
        # reference against which the HBM byte counters are scaled
        log("bench: copy calibration")
        B = torch.empty_like(A)
        B.copy_(A)
        torch.cuda.synchronize()
        del B

    # read-only ceiling on the same buffer (torch reduction, measurement only)
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    for _ in range(10):
        s = A.sum()
    torch.cuda.synchronize()
    read_gbs = bytes_a * 10 / (time.perf_counter() - tr0) / 1e9
    del s

    traffic = _traffic("traffic_fused_fp32_sketch_2p20x1024.json", ["apply_fp32.hip"], alg_bytes)
    out = {
        "metric": "block-SRHT sketch GB/s of A (FP32 fused apply)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
        "read_ceiling_GBs": round(read_gbs, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "fused_fp32_kernel<64>",
                     "kernel_avg_us": round(kern_avg_ms * 1e3, 2),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if not args.skip_cpu_baseline:
        log("bench: timing the CPU oracle on one block")
        out["cpu_baseline"] = cpu_baseline(A, cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
