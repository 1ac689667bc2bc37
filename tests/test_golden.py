"""The golden plan fixtures are what the oracle produces (regenerable, cited)."""
import json
import os

import numpy as np
import pytest

from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("fx", make_golden.FIXTURES, ids=[f[0] for f in make_golden.FIXTURES])
def test_golden_reproducible(fx):
    name, *args = fx
    with open(os.path.join(HERE, name + ".json")) as f:
        doc = json.load(f)
    fresh = make_golden.make(name, *args)
    for key in ("R", "Dbits", "Dtbits"):
        assert doc[key] == fresh[key]
    if "omega" in doc:
        assert np.allclose(np.array(doc["omega"]), np.array(fresh["omega"]), rtol=0, atol=1e-15)
        om = np.array(doc["omega"])
        assert np.allclose(np.abs(om), 1 / np.sqrt(doc["l"]), atol=1e-15)
