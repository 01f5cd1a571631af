"""The oracle's result on the 1000 x 32^3 workload is stable: the stored
fingerprint was written by tests/golden/make_golden.py (oracle + seeded
inputs only).  A change here means the oracle or the input generator moved."""
import json
import os

from tests.golden.make_golden import config1_result, fingerprint

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_config1_fingerprint():
    with open(os.path.join(HERE, "config1_oracle.json")) as f:
        want = json.load(f)
    got = fingerprint(config1_result())
    assert got["sha256"] == want["sha256"]
    assert got["frobenius_first8"] == want["frobenius_first8"]
