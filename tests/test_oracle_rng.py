"""Pins of the oracle's counter-based generator and plan tables.

The generator is pinned to numpy.random.Philox, an independent library
implementation of Philox4x64-10 (numpy pre-increments its counter, so its
first block for counter c is philox(c + 1)).  The Fisher-Yates sampler is
pinned to a plain dense-array implementation.
"""
import numpy as np
import pytest

from oracle import rng


def _numpy_block(counter, key):
    c = list(counter)
    # numpy generates philox(counter + 1) first: step the counter back by one
    for w in range(4):
        if c[w] > 0:
            c[w] -= 1
            break
        c[w] = rng.MASK64
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (12345, 0)),
    ((5, 7, rng.TAG_D, 0), (0xDEADBEEFCAFEF00D, 0)),
    ((2 ** 64 - 1, 3, rng.TAG_R, 0), (42, 0)),
    ((123456789, 2 ** 40, rng.TAG_DT, 9), (2 ** 64 - 1, 77)),
])
def test_philox_matches_numpy(counter, key):
    assert rng.philox4x64(counter, key) == _numpy_block(counter, key)


def test_sign_bit_order():
    seed = 99
    bits = rng.sign_bits(600, 3, rng.TAG_D, seed)
    for x in [0, 1, 63, 64, 200, 255, 256, 511, 599]:
        words = _numpy_block((x // 256, 3, rng.TAG_D, 0), (seed, 0))
        b = x % 256
        assert bits[x] == (words[b // 64] >> (b % 64)) & 1


def test_signs_balanced():
    bits = rng.sign_bits(1 << 16, 0, rng.TAG_D, 7)
    frac = bits.mean()
    assert abs(frac - 0.5) < 6 * 0.5 / np.sqrt(1 << 16)


def test_rows_with_replacement_uniform():
    r, l = 16, 16000
    R = rng.sample_rows(r, l, 5)
    assert R.min() >= 0 and R.max() < r
    counts = np.bincount(R, minlength=r)
    chi2 = float(np.sum((counts - l / r) ** 2 / (l / r)))
    assert chi2 < 50.0  # 15 dof; p(chi2 > 50) ~ 1e-5
    words = [_numpy_block((j, 0, rng.TAG_R, 0), (5, 0))[0] for j in range(20)]
    assert list(R[:20]) == [w % r for w in words]


def _dense_fisher_yates(r, l, seed):
    pool = list(range(r))
    out = []
    for j in range(l):
        u = _numpy_block((j, 0, rng.TAG_R, 0), (seed, 0))[0]
        t = j + (u * (r - j) >> 64)
        pool[j], pool[t] = pool[t], pool[j]
        out.append(pool[j])
    return out


@pytest.mark.parametrize("r,l", [(8, 8), (64, 17), (1024, 1024), (4096, 100)])
def test_rows_without_replacement(r, l):
    R = rng.sample_rows(r, l, 11, rng.WITHOUT_REPLACEMENT)
    assert list(R) == _dense_fisher_yates(r, l, 11)
    assert len(set(R.tolist())) == l
    if l == r:
        assert sorted(R.tolist()) == list(range(r))


def test_without_replacement_needs_l_le_r():
    with pytest.raises(ValueError):
        rng.sample_rows(8, 9, 0, rng.WITHOUT_REPLACEMENT)


def test_plan_validation():
    pl = rng.Plan(12, 1, 4, 0)     # r = 12: a partial SRHT padded to 16
    assert pl.rp == 16 and np.all(pl.R < 16)
    with pytest.raises(ValueError):
        rng.Plan(12, 2, 10, 0, rng.WITHOUT_REPLACEMENT)   # r = 6, r' = 8 < l
    with pytest.raises(ValueError):
        rng.Plan(16, 3, 4, 0)      # p does not divide n
    with pytest.raises(ValueError):
        rng.Plan(16, 2, 17, 0)     # l > n


def test_subsample_keying():
    """A p = 1 plan on the first r rows reproduces block 0 of a p-block plan."""
    big = rng.Plan(4 * 256, 4, 96, 2024)
    small = rng.Plan(256, 1, 96, 2024)
    assert np.array_equal(big.R, small.R)
    assert np.array_equal(big.D[0], small.D[0])
    assert np.array_equal(big.Dt[0], small.Dt[0])
    assert not np.array_equal(big.D[0], big.D[1])
