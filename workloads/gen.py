"""Seeded input generators (no method arithmetic).  See the package docstring."""

import math

import numpy as np
import torch

SPECTRA = {
    "inv": lambda j: j ** -1.0,             # s_j = j^-1
    "inv_sq": lambda j: j ** -2.0,          # s_j = j^-2
    "exp64": lambda j: torch.exp(-j / 64.0),  # s_j = exp(-j/64)
    "pow1.5": lambda j: j ** -1.5,           # s_j = j^-1.5
    "cube": lambda j: j ** -3.0,             # s_j = j^-3
}

# The five workloads: sizes and recipes (the first is the small case the
# oracle finishes in seconds; the others are the full-size cases).
CONFIGS = {
    "c1_rsvd_small": dict(n=4096, m=256, p=4, l=128, k=50, spectrum="inv_sq", seed=0),
    "c2_fp32_apply": dict(n=1 << 20, m=1024, p=16, l=512, k=256, spectrum="exp64", seed=0),
    "c3_split_bf16": dict(n=1 << 20, m=1024, p=16, l=512, k=256, spectrum="exp64", seed=0),
    "c5_nystrom": dict(n=65536, d=4096, p=64, l=1024, k=512, spectrum="cube", seed=0),
    # The large sketch workload in the orientation of Algorithm 1: the
    # transpose (m x n, row-major) of the 2^20 x 1024 input, sketched from the
    # right along its contiguous dimension.
    "right_apply_large": dict(n=1 << 20, m=1024, p=16, l=512, spectrum="exp64", seed=0),
}


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def haar(m, seed, device="cpu"):
    """Haar-random m x m orthogonal matrix (float64): QR of a Gaussian,
    columns multiplied by sign(diag(R))."""
    g = _gen(seed, device)
    G = torch.randn(m, m, generator=g, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(G)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def _spectrum(name, m, device):
    j = torch.arange(1, m + 1, dtype=torch.float64, device=device)
    return SPECTRA[name](j)


def lowrank_tall(n, m, spectrum, seed, device="cpu", row_chunk=1 << 16):
    """A = X diag(s) W^T (n x m float32), X Gaussian / sqrt(n), W Haar.

    X is drawn in row chunks from one generator (seed), W from seed + 1.
    """
    s = _spectrum(spectrum, m, device)
    W = haar(m, int(seed) + 1, device)
    SWt = (s[:, None] * W.T).contiguous()
    g = _gen(seed, device)
    A = torch.empty(n, m, dtype=torch.float32, device=device)
    scale = 1.0 / math.sqrt(n)
    for r0 in range(0, n, row_chunk):
        r1 = min(n, r0 + row_chunk)
        X = torch.randn(r1 - r0, m, generator=g, dtype=torch.float64, device=device)
        A[r0:r1] = ((X * scale) @ SWt).to(torch.float32)
    return A


def spd(n, d, spectrum, seed, device="cpu", return_factors=False, shift=0.0):
    """A = X diag(s) X^T + shift I (n x n float32), X = orth(Gaussian n x d)."""
    g = _gen(seed, device)
    G = torch.randn(n, d, generator=g, dtype=torch.float64, device=device)
    X, _ = torch.linalg.qr(G)
    s = _spectrum(spectrum, d, device)
    A = (X * s[None, :]) @ X.T
    if shift:
        A.diagonal().add_(float(shift))
    A = (0.5 * (A + A.T)).to(torch.float32)  # exactly symmetric after rounding
    if return_factors:
        return A, X, s
    return A


def gaussian_cols(n, m, spectrum, seed, device="cpu"):
    """A = X diag(s) (n x m float32), X ~ N(0, 1)."""
    g = _gen(seed, device)
    s = _spectrum(spectrum, m, device).to(torch.float32)
    X = torch.randn(n, m, generator=g, dtype=torch.float32, device=device)
    return X * s[None, :]


def gaussian_rows(m, n, spectrum, seed, device="cpu"):
    """A = diag(s) X (m x n float32), X ~ N(0, 1): gaussian_cols transposed in
    shape, for inputs sketched along their rows."""
    g = _gen(seed, device)
    s = _spectrum(spectrum, m, device).to(torch.float32)
    X = torch.randn(m, n, generator=g, dtype=torch.float32, device=device)
    return s[:, None] * X


def serving_jobs(count, rate, seed):
    """Job descriptors of the serving workload: Poisson arrivals at `rate`/s.

    n = 2^a, a ~ U{14..20}; m = round(exp(U[ln 64, ln 2048])); p ~ U{1,4,16,64};
    k ~ U{16..256}; l = 2k + 32; payload seed per job.
    """
    rs = np.random.default_rng(seed)
    t = np.cumsum(rs.exponential(1.0 / rate, size=count))
    jobs = []
    for i in range(count):
        a = int(rs.integers(14, 21))
        m = int(round(math.exp(rs.uniform(math.log(64), math.log(2048)))))
        p = int(rs.choice([1, 4, 16, 64]))
        k = int(rs.integers(16, 257))
        jobs.append(dict(id=i, arrival=float(t[i]), n=1 << a, m=m, p=p, k=k,
                         l=2 * k + 32, seed=int(rs.integers(0, 2 ** 63))))
    return jobs
