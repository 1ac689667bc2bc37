"""Counter-based RNG and the block SRHT tables (oracle side; test infrastructure).

The paper only says that each processor's Omega^(i) comes from a seeded random
generator (section 4.1 and 4.2).  Bit-exact agreement between this oracle and
the GPU library therefore needs a written generator specification.  This
module is the oracle's independent implementation of that specification:

Generator
  Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11), 4 x 64-bit counter, 2 x 64-bit key, 10 rounds.
  key = (seed mod 2**64, 0).  One call yields four 64-bit words w0..w3, read
  as a 256-bit string in which bit b is bit (b % 64) of word b // 64.

Streams (tag in counter word 2)
  TAG_R  = 1   row sample R (shared by all p blocks, eq. (2.3))
  TAG_D  = 2   input signs D^(i)  (r x r diagonal per block)
  TAG_DT = 3   output signs Dt^(i) (l x l diagonal per block)

Tables
  D^(i)_x   = bit (x % 256) of philox((x // 256, i, TAG_D, 0));  bit 0 -> +1
  Dt^(i)_j  = bit (j % 256) of philox((j // 256, i, TAG_DT, 0)); bit 1 -> -1
  R_j, with replacement (the block SRHT default, section 2):
            = w0(philox((j, 0, TAG_R, 0))) mod r     (r is a power of two)
  R_j, without replacement (allowed for the SRHT, eq. (2.1)):
            partial Fisher-Yates over pool = [0, r): for j = 0 .. l-1,
            u = w0(philox((j, 0, TAG_R, 0))),
            t = j + floor(u * (r - j) / 2**64), swap(pool[j], pool[t]),
            R_j = pool[j].
  Rows of Omega are kept in draw order j = 0 .. l-1 (not sorted).

Keying by (seed, block, index) makes a p = 1 plan with the same r and seed
reproduce block 0 of any plan: the 2**16-row subsample check relies on it.

Blocks whose size r is not a power of two (section 2: a partial SRHT, the
first r columns of an SRHT of size r' = the next power of two, i.e. the input
block padded with zeros to r' rows).  R is drawn from [0, r') and D^(i) holds
the first r entries of block i's stream, so a plan with such an r equals the
power-of-two plan (p r', p) on the input with r' - r zero rows appended to
every block.

The oracle's Philox is checked against numpy.random.Philox, an independent
library implementation of the same published generator.
"""

import numpy as np

MASK64 = (1 << 64) - 1

# Philox4x64 round multipliers and Weyl key increments (SC'11, table of
# recommended constants for the 4x64 variant).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
PHILOX_ROUNDS = 10

TAG_R = 1
TAG_D = 2
TAG_DT = 3

WITH_REPLACEMENT = 0
WITHOUT_REPLACEMENT = 1


def philox4x64(counter, key, rounds=PHILOX_ROUNDS):
    """One Philox4x64 block: 4 x 64-bit counter, 2 x 64-bit key -> 4 words.

    Each round multiplies words 0 and 2 by the two constants, keeps the
    128-bit products' high and low halves, mixes them with words 1, 3 and the
    key, and the key is bumped by the Weyl constants between rounds.
    """
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for _ in range(rounds):
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & MASK64
        k1 = (k1 + PHILOX_W1) & MASK64
    return (x0, x1, x2, x3)


def _bits256(words):
    """The four output words as a 256-entry 0/1 array, bit b = word b//64."""
    raw = np.array(words, dtype="<u8").tobytes()
    return np.unpackbits(np.frombuffer(raw, dtype=np.uint8), bitorder="little")


def sign_bits(count, block, tag, seed):
    """Bits 0..count-1 of the (block, tag) sign stream, 1 meaning -1."""
    key = (seed, 0)
    nwords = (count + 255) // 256
    bits = np.concatenate(
        [_bits256(philox4x64((c, block, tag, 0), key)) for c in range(nwords)]
    ) if nwords else np.zeros(0, dtype=np.uint8)
    return bits[:count].copy()


def signs_from_bits(bits):
    """Rademacher values from bits: 0 -> +1.0, 1 -> -1.0 (float64)."""
    return 1.0 - 2.0 * np.asarray(bits, dtype=np.float64)


def sample_rows(r, l, seed, sampling=WITH_REPLACEMENT):
    """The shared row sample R of eq. (2.3): l indices in [0, r), draw order."""
    key = (seed, 0)
    words = [philox4x64((j, 0, TAG_R, 0), key)[0] for j in range(l)]
    if sampling == WITH_REPLACEMENT:
        return np.array([w % r for w in words], dtype=np.int64)
    if sampling != WITHOUT_REPLACEMENT:
        raise ValueError("unknown sampling mode")
    if l > r:
        raise ValueError("sampling without replacement needs l <= r")
    pool = {}  # sparse Fisher-Yates: only touched slots are stored

    def get(i):
        return pool.get(i, i)

    out = np.empty(l, dtype=np.int64)
    for j, u in enumerate(words):
        t = j + ((u * (r - j)) >> 64)
        pj, pt = get(j), get(t)
        pool[j], pool[t] = pt, pj
        out[j] = pool[j]
    return out


class Plan:
    """The random tables of one block SRHT Omega (l x n), eq. (2.3).

    n rows of the sketched matrix split into p blocks of r = n/p rows each,
    each padded with zeros to rp = the next power of two >= r (rp = r when r
    is a power of two: no padding).  Holds
      R   : (l,)   int64 sample indices in [0, rp), shared by all blocks
      D   : (p, r) float64 +-1, input signs D^(i) of the r real rows
      Dt  : (p, l) float64 +-1, output signs Dt^(i)
    plus the raw 0/1 bits, for comparison with tables exported by the GPU
    library.
    """

    def __init__(self, n, p, l, seed, sampling=WITH_REPLACEMENT):
        n, p, l = int(n), int(p), int(l)
        if p < 1 or n < 1 or n % p:
            raise ValueError("p must divide n")
        r = n // p
        rp = 1 << (r - 1).bit_length()
        if not 1 <= l <= n:
            raise ValueError("need 1 <= l <= n")
        self.n, self.p, self.l, self.r, self.rp = n, p, l, r, rp
        self.seed = int(seed) & MASK64
        self.sampling = sampling
        self.R = sample_rows(rp, l, self.seed, sampling)
        self.D_bits = np.stack([sign_bits(r, i, TAG_D, self.seed) for i in range(p)])
        self.Dt_bits = np.stack([sign_bits(l, i, TAG_DT, self.seed) for i in range(p)])
        self.D = signs_from_bits(self.D_bits)
        self.Dt = signs_from_bits(self.Dt_bits)
