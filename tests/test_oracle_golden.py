"""The oracle against its stored results (tests/golden/oracle_golden.json, written by
tests/golden/make_oracle_golden.py from oracle/ alone): a later change to the oracle's
arithmetic shows up here and must name the passage of the paper that justifies it
before the fixture is rewritten."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def _flat(d, prefix=""):
    for k, v in d.items():
        if isinstance(v, dict):
            yield from _flat(v, prefix + k + ".")
        else:
            yield prefix + k, v


@pytest.fixture(scope="module")
def fresh(oracle_lib):
    import make_oracle_golden
    return make_oracle_golden.compute()


@pytest.mark.parametrize("case", ["tiny_cube", "mixed_body", "rigid_box", "silhouette"])
def test_oracle_matches_stored_results(fresh, case):
    with open(os.path.join(HERE, "golden", "oracle_golden.json")) as fh:
        stored = json.load(fh)[case]
    got = dict(_flat(fresh[case]))
    for k, v in _flat(stored):
        a, b = np.asarray(got[k], np.float64), np.asarray(v, np.float64)
        assert a.shape == b.shape, k
        assert np.allclose(a, b, rtol=1e-9, atol=1e-14), (case, k, np.abs(a - b).max())
