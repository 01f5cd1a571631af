"""Writes the oracle fingerprints under tests/golden/.  Calls only the CPU
oracle and the seeded input generator; no value here comes from the GPU path.

    python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2203_09353_amd import inputs  # noqa: E402


def config1_result():
    """1000 instances of 32x32x32, alpha = 1, beta = 0, A and B uniform[-1, 1)
    from seed 0 (streams 0 and 1); C starts as NaN and must not be read."""
    batch, m = 1000, 32
    A = inputs.uniform_batch(0, 0, batch, m, m).numpy()
    B = inputs.uniform_batch(0, 1, batch, m, m).numpy()
    C = np.full((batch, m, m), np.nan)
    oracle.gemm_batched("N", "N", m, m, m, 1.0, A, B, 0.0, C)
    return C


def fingerprint(C):
    return {
        "sha256": hashlib.sha256(np.ascontiguousarray(C).tobytes()).hexdigest(),
        "sum": float(np.sum(C)),
        "frobenius_first8": [float(np.linalg.norm(C[i])) for i in range(8)],
    }


if __name__ == "__main__":
    out = {
        "workload": "1000 x (32x32x32) FP64, alpha=1, beta=0, uniform[-1,1) seed 0",
        "definition": "Eq. 1 (Section II) via the CPU oracle",
        **fingerprint(config1_result()),
    }
    with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["sha256"])
