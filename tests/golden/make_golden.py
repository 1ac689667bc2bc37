"""Write the golden plan fixtures under tests/golden/ from the oracle only.

Each fixture is a small block SRHT plan (eq. (2.3)): its row sample R, the
sign bits of D and Dt packed the way the C ABI exports them (bit g%32 of
word g/32), and Omega formed explicitly from the closed form.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import rng, sketch  # noqa: E402

FIXTURES = [
    # name, n, p, l, seed, sampling
    ("plan_n16_p2_l6", 16, 2, 6, 20221020, rng.WITH_REPLACEMENT),
    ("plan_n64_p1_l64_perm", 64, 1, 64, 7, rng.WITHOUT_REPLACEMENT),
    ("plan_n40_p40_l5_r1", 40, 40, 5, 3, rng.WITH_REPLACEMENT),
    ("plan_n1024_p4_l128", 1024, 4, 128, 0, rng.WITH_REPLACEMENT),
]


def pack_bits(bits):
    bits = np.asarray(bits, dtype=np.uint64).ravel()
    words = np.zeros((len(bits) + 31) // 32, dtype=np.uint64)
    for g, b in enumerate(bits):
        words[g // 32] |= b << np.uint64(g % 32)
    return [int(w) for w in words]


def make(name, n, p, l, seed, sampling):
    plan = rng.Plan(n, p, l, seed, sampling)
    lw = (l + 31) // 32
    dt_words = []
    for i in range(p):
        row = np.zeros(lw * 32, dtype=np.uint8)
        row[:l] = plan.Dt_bits[i]
        dt_words += pack_bits(row)
    doc = {
        "n": n, "p": p, "l": l, "seed": seed, "sampling": sampling,
        "R": [int(v) for v in plan.R],
        "Dbits": pack_bits(plan.D_bits.ravel()),
        "Dtbits": dt_words,
    }
    if n <= 64:
        doc["omega"] = sketch.omega_explicit(plan).tolist()
    return doc


if __name__ == "__main__":
    for name, *args in FIXTURES:
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(make(name, *args), f, indent=0)
            f.write("\n")
        print("wrote", name)
