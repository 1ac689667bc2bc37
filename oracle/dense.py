"""Dense Gaussian and Rademacher sketches Y = G A in FP64: the embeddings the
block SRHT is compared with in section 4.  Oracle side; test infrastructure.

The paper does not fix a generator for them.  Reading: the same Philox4x64-10
as the block SRHT tables, key (seed, 0), so that both sides draw G from one
published definition:
  Gaussian   G[j, x] = z / sqrt(l).  Counter (x >> 3, j, 4, 0); of the four
             64-bit output words, word q = (x & 7) >> 1 gives
             u1 = (lo + 1/2) 2^-32 from its low and u2 = (hi + 1/2) 2^-32 from
             its high 32 bits; with rho = sqrt(-2 ln u1) the Box-Muller
             transform (Box and Muller, 1958) gives z = rho cos(2 pi u2) for
             even x and z = rho sin(2 pi u2) for odd x.
  Rademacher G[j, x] = +-1 / sqrt(l): bit (x & 255) of the 256-bit output for
             counter (x >> 8, j, 5, 0), bit 1 -> -1 (the sign stream of the
             block SRHT's D tables with tag 5).
"""

import numpy as np

from .rng import philox4x64, sign_bits, signs_from_bits

TAG_GAUSS = 4
TAG_RADEMACHER = 5
GAUSSIAN = 0
RADEMACHER = 1


def gaussian_words(seed, j, n):
    """The (n + 7) // 8 Philox outputs of row j, as an array of 64-bit words
    (shape ((n + 7) // 8, 4))."""
    key = (int(seed), 0)
    return np.array([philox4x64((c, j, TAG_GAUSS, 0), key) for c in range((n + 7) // 8)],
                    dtype=np.uint64)


def box_muller(words):
    """Eight normals per output (rows of `words`): for each word q, the pair
    (rho cos(2 pi u2), rho sin(2 pi u2)) from its low / high 32-bit halves."""
    lo = (words & np.uint64(0xFFFFFFFF)).astype(np.float64)
    hi = (words >> np.uint64(32)).astype(np.float64)
    u1 = (lo + 0.5) * 2.0 ** -32
    u2 = (hi + 0.5) * 2.0 ** -32
    rho = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(words.shape + (2,))
    z[..., 0] = rho * np.cos(2.0 * np.pi * u2)
    z[..., 1] = rho * np.sin(2.0 * np.pi * u2)
    return z.reshape(words.shape[0], 8)


def gaussian_row(seed, j, n, l):
    return box_muller(gaussian_words(seed, j, n)).ravel()[:n] / np.sqrt(l)


def rademacher_row(seed, j, n, l):
    return signs_from_bits(sign_bits(n, j, TAG_RADEMACHER, seed)) / np.sqrt(l)


def omega(kind, seed, l, n):
    """G (l x n, float64)."""
    row = gaussian_row if kind == GAUSSIAN else rademacher_row
    return np.stack([row(seed, j, n, l) for j in range(l)])


def dense_sketch(kind, seed, l, A):
    """Y = G A (l x m, float64)."""
    A = np.asarray(A, dtype=np.float64)
    return omega(kind, seed, l, A.shape[0]) @ A
