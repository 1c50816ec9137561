"""The oracle still reproduces its committed regression record."""
import json
import os

import numpy as np

from tests.golden.make_golden import abc16

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_abc16_regression():
    with open(os.path.join(HERE, "oracle_abc16_10steps.json")) as f:
        ref = json.load(f)
    got = abc16()
    for k, v in ref["diag"].items():
        assert abs(got["diag"][k] - v) <= 1e-12 * max(1.0, abs(v)), k
    assert np.allclose(got["field_rms"], ref["field_rms"], rtol=1e-12, atol=0)
    assert np.allclose(got["probe_z3_y5_x7"], ref["probe_z3_y5_x7"], rtol=1e-11, atol=1e-15)
