"""Regression guard: the oracle reproduces its stored 20-step trajectory
(written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

from golden.make_golden import trajectory


def test_oracle_matches_stored_trajectory():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "oracle_diamond16_20steps.json")) as f:
        ref = json.load(f)
    got = trajectory()
    J, Jr = np.array(got["J"]), np.array(ref["J"])
    assert np.max(np.abs(J - Jr)) < 1e-12 * np.max(np.abs(Jr))
    assert abs(got["energy_end"] - ref["energy_end"]) < 1e-10
    assert abs(got["rho_sum_end"] - ref["rho_sum_end"]) < 1e-10
