"""The oracle against its stored regression summaries (tests/golden/).

These values were written by tests/golden/make_golden.py, which calls only
the oracle and the scene generator.  They guard the oracle against silent
changes; the pins in test_oracle_pins.py are what tie it to the paper.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_golden as G  # noqa: E402

with open(os.path.join(HERE, "golden", "oracle_regression.json")) as f:
    STORED = json.load(f)


@pytest.mark.parametrize("case", G.CASES, ids=[c[0] for c in G.CASES])
def test_oracle_matches_stored_summary(case):
    ref = next(s for s in STORED if s["name"] == case[0])
    got = G.summarize(*case)
    assert got["inputs_sha256_16"] == ref["inputs_sha256_16"], "scene generator changed"
    for key in ("d_idx_histogram", "d_idx_sha256_16", "q_static_count", "holes"):
        assert got[key] == ref[key], key
    # sums of FP64 values; OpenMP may change the order of the per-iteration sum
    np.testing.assert_allclose(got["L_sum"], ref["L_sum"], rtol=1e-12)
    for key in ("q_sum", "rho_sum", "rgb_sum", "beta"):
        assert got[key] == pytest.approx(ref[key], rel=1e-12), key
