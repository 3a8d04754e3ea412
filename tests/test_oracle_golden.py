"""Regression pin: the oracle still produces the stored small fixtures
(written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_fuse_small.json")


def test_oracle_matches_stored_fixtures(oracle):
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    assert len(cases) >= 4
    for c in cases:
        out = oracle.fuse(c["wavelet"], np.array(c["pan"], float), np.array(c["ms"], float), c["gain"])
        ref = np.array([[[float(v) for v in row] for row in band] for band in c["out"]])
        assert out.shape == ref.shape
        assert np.abs(out - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
