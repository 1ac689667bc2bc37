"""The large sketch workload checked in full against the FP64 oracle
(section 2, eq. (2.3)-(2.4)): A is 2^20 x 1024 FP32 (A = X diag(exp(-j/64))
W^T, seed 0), p = 16 blocks of r = 65536 rows, l = 512 samples with
replacement.  All 512 x 1024 outputs of the FP32 sketch and of the split-BF16
sketch (the same plan seed) are compared with the oracle's FP64 sketch of the
same FP32 input, computed once per module (sketch_parallel, bitwise the
oracle's sketch; about half a minute on the host):
relative Frobenius error of the whole Y and of every 64-column tile (the
kernels' column tile), and the largest entry error relative to max |Y|.
Bounds: 1e-5 (FP32) and 1e-4 (split-BF16) for each.

The launch that produces Y is the one the benchmark times (same plan, same
input shape), so every workgroup tile, row split and the XCD-remapped tile
order of that launch is covered.
"""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import rng, sketch
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu

TILE = 64


@pytest.fixture(scope="module")
def full_case():
    dev = device()
    cfg = workloads.CONFIGS["c2_fp32_apply"]
    n, m, p, l, seed = cfg["n"], cfg["m"], cfg["p"], cfg["l"], cfg["seed"]
    say("full size input", n, m, p, l)
    A = workloads.lowrank_tall(n, m, cfg["spectrum"], seed, device=dev)
    torch.cuda.synchronize()
    say("oracle sketch of the full input (FP64)")
    Y_ref = sketch.sketch_parallel(rng.Plan(n, p, l, seed), A.cpu().numpy(), workers=8)
    yield A, Y_ref, cfg
    del A


def _check(Y, Y_ref, tol, what):
    Yh = to64(Y)
    D = Yh - Y_ref
    err = float(np.linalg.norm(D) / np.linalg.norm(Y_ref))
    worst_tile = 0.0
    for c0 in range(0, Y_ref.shape[1], TILE):
        t = float(np.linalg.norm(D[:, c0:c0 + TILE]) / np.linalg.norm(Y_ref[:, c0:c0 + TILE]))
        worst_tile = max(worst_tile, t)
    emax = float(np.max(np.abs(D)) / np.max(np.abs(Y_ref)))
    say(f"  {what}: rel fro {err:.3e}, worst tile {worst_tile:.3e}, max entry {emax:.3e}")
    assert np.all(np.isfinite(Yh))
    assert err <= tol
    assert worst_tile <= tol
    assert emax <= tol


def test_full_size_fp32(full_case):
    A, Y_ref, cfg = full_case
    plan = bs.Plan(cfg["n"], cfg["p"], cfg["l"], cfg["seed"], device=A.device)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    _check(Y, Y_ref, 1e-5, "fp32")


def test_full_size_split_bf16(full_case):
    A, Y_ref, cfg = full_case
    plan = bs.Plan(cfg["n"], cfg["p"], cfg["l"], cfg["seed"], precision=bs.SPLIT_BF16,
                   device=A.device)
    Y = bs.bsrht_apply(plan, A)
    torch.cuda.synchronize()
    _check(Y, Y_ref, 1e-4, "split-bf16")
