"""Plain FP64 CPU oracle for the block SRHT sketch, randomized SVD and Nystrom.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links this package; only the tests, the
smoke check of the entry module and the CPU-baseline leg of the benchmark may.
It shares no code with the HIP path: the counter-based generator, the tables,
the Walsh-Hadamard transform and the low-rank algorithms are written here
independently, in plain numpy/scipy, from the paper's definitions.

Modules
  rng      Philox4x64-10 (Salmon et al., SC'11) and the sign/sample tables
           of the block SRHT (section 2, eq. (2.3)).
  sketch   Omega formed explicitly from its closed form, and Omega @ A by
           per-block FWHT + subsample + signs + sum (section 2, eq. (2.4)).
  lowrank  Algorithm 1 (RSVD) and Algorithm 2 (Nystrom), section 3.
  single_view  Algorithm 3 (single-view RSVD), section 3.3.
  dense    Gaussian and Rademacher comparison sketches (section 4) from
           the same Philox stream.
  metrics  relative errors used by the parity tests.

Every function cites the passage it follows.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""

from . import rng, sketch, lowrank, metrics  # noqa: F401
