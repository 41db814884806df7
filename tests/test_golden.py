"""The stored tiny-workload oracle output (tests/golden, written by tests/golden/make_golden.py from the
oracle alone) is reproduced by the oracle: guards the oracle and the input generators against drift."""
import json
import os

import numpy as np

from tests.golden import make_golden

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tiny_er_n200_golden_reproduced():
    with open(os.path.join(HERE, "tiny_er_n200_oracle.json")) as f:
        stored = json.load(f)
    now = make_golden.tiny_er_n200()
    assert now["topk"] == stored["topk"] and now["targets"] == stored["targets"]
    assert abs(now["log_scale"] - stored["log_scale"]) < 1e-12
    s0, s1 = np.array(stored["scores"]), np.array(now["scores"])
    assert np.max(np.abs(s0 - s1)) / np.max(np.abs(s0)) < 1e-13
