"""GPU parity of the dense comparison sketches Y = G A (Gaussian and
Rademacher G from the block SRHT's Philox stream; section 4's baseline)
against the FP64 oracle, through the C ABI.

G itself (A = I): Rademacher entries bit-exact, Gaussian entries within one
FP32 ulp (both sides evaluate Box-Muller in FP64 and round once).  Y = G A
within 1e-5 relative Frobenius error (FP32 products accumulated over splits
of the n-long contraction, summed in FP64)."""
import numpy as np
import pytest
import torch

import paper_2210_11295_amd as bs
import workloads
from oracle import dense, metrics
from tests.gpu_util import device, to64, say

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.mark.parametrize("kind", [bs.DENSE_GAUSSIAN, bs.DENSE_RADEMACHER])
@pytest.mark.parametrize("n,l", [(1024, 64), (1000, 17)])
def test_dense_omega_entries(kind, n, l):
    dev = device()
    say("dense omega", kind, n, l)
    I = torch.eye(n, dtype=torch.float32, device=dev)
    G = to64(bs.bsrht_dense_sketch(kind, 21, l, I))
    Go = dense.omega(kind, 21, l, n).astype(np.float32).astype(np.float64)
    if kind == bs.DENSE_RADEMACHER:
        assert np.array_equal(G, Go)
    else:
        assert np.all(np.abs(G - Go) <= 2.0 ** -23 * np.abs(Go) + 1e-30)


@pytest.mark.parametrize("kind", [bs.DENSE_GAUSSIAN, bs.DENSE_RADEMACHER])
@pytest.mark.parametrize("n,m,l", [(4096, 100, 64), (1000, 33, 17), (8192, 256, 200)])
def test_dense_sketch_parity(kind, n, m, l):
    dev = device()
    say("dense sketch", kind, n, m, l)
    A = workloads.gaussian_cols(n, m, "inv_sq", 3, device=dev)
    Y = bs.bsrht_dense_sketch(kind, 5, l, A)
    torch.cuda.synchronize()
    err = metrics.rel_fro(to64(Y), dense.dense_sketch(kind, 5, l, to64(A)))
    say("  rel err", err)
    assert err <= TOL


def test_dense_repeatable_and_errors():
    dev = device()
    A = workloads.gaussian_cols(4096, 64, "inv_sq", 1, device=dev)
    Y1 = bs.bsrht_dense_sketch(bs.DENSE_GAUSSIAN, 2, 128, A).clone()
    Y2 = bs.bsrht_dense_sketch(bs.DENSE_GAUSSIAN, 2, 128, A)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    L = bs.lib()
    Y = torch.zeros(8, 64, device=dev)
    ws = torch.zeros(16, dtype=torch.uint8, device=dev)
    P = bs._ptr
    assert L.bsrht_dense_sketch(7, 0, 4096, 8, P(A), 64, 64, P(Y), 64, P(ws), 16, None) == -1
    assert L.bsrht_dense_sketch(0, 0, 4096, 8, P(A), 0, 64, P(Y), 64, P(ws), 16, None) == 0
    assert L.bsrht_dense_sketch(0, 0, 4096, 8, P(A), 64, 63, P(Y), 64, P(ws), 16, None) == -1
    assert L.bsrht_dense_sketch(0, 0, 4096, 8, P(A), 64, 64, P(Y), 64, P(ws), 16, None) == -2
    assert L.bsrht_dense_workspace(0, 8, 64) == 0


def test_dense_full_size_sampled_entries():
    """The 2^20 x 1024 input, l = 512 (the launch the benchmark times):
    sampled rows of G from the oracle, dotted with sampled columns of A."""
    dev = device()
    cfg = workloads.CONFIGS["c2_fp32_apply"]
    n, m, l, seed = cfg["n"], cfg["m"], cfg["l"], cfg["seed"]
    A = workloads.lowrank_tall(n, m, cfg["spectrum"], seed, device=dev)
    Y = to64(bs.bsrht_dense_sketch(bs.DENSE_GAUSSIAN, seed + 7, l, A))
    rs = np.random.default_rng(3)
    rows = rs.choice(l, 3, replace=False)
    cols = rs.choice(m, 5, replace=False)
    Ac = to64(A[:, torch.as_tensor(cols, device=dev)])
    diff = ref = 0.0
    for j in rows:
        g = dense.gaussian_row(seed + 7, int(j), n, l)
        y = g @ Ac
        diff += float(np.sum((Y[j, cols] - y) ** 2))
        ref += float(np.sum(y ** 2))
    err = np.sqrt(diff / ref)
    say("  sampled rel err", err)
    assert err <= TOL
