"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This package holds no part of the block SRHT, RSVD or Nystrom arithmetic:
only the matrices those methods are applied to.  Both the oracle-side tests
and the GPU-side calls take their inputs from here, so a parity test always
feeds the same tensor to both sides.

Recipes (seeded; torch generators, float64 formation, one rounding to float32)
  lowrank_tall(n, m, spectrum, seed):  A = X diag(s) W^T,
      X ~ N(0,1)^{n x m} / sqrt(n), W Haar-random m x m orthogonal
      (QR of a Gaussian with the signs of diag(R) folded in, Mezzadri 2007),
      s_j = spectrum(j), j = 1..m.
  spd(n, d, spectrum, seed, shift=0):  A = X diag(s) X^T + shift I,
      X = orth(N(0,1)^{n x d}).
  gaussian_cols(n, m, spectrum, seed):  A = X diag(s) with X ~ N(0,1)
      (the serving payload; W = I).
  gaussian_rows(m, n, spectrum, seed):  A = diag(s) X with X ~ N(0,1)
      (inputs sketched along their rows).
"""

from .gen import (SPECTRA, lowrank_tall, spd, gaussian_cols, gaussian_rows,  # noqa: F401
                  haar, CONFIGS, serving_jobs)
