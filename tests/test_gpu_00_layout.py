"""Pins the lane layout of v_mfma_f64_16x16x4_f64 that the GEMM kernels
assume, on the device, with small integers (exact)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_mfma_lane_layout():
    """Pins the lane layout the kernels assume for v_mfma_f64_16x16x4_f64:
    lane l holds A(l%16, l/16), B(l/16, l%16) and D(l/16 + 4v, l%16)."""
    from paper_2203_09353_amd import microbench
    rng = np.random.default_rng(0)
    Am = rng.integers(-8, 9, (16, 4)).astype(float)
    Bm = rng.integers(-8, 9, (4, 16)).astype(float)
    Cm = rng.integers(-8, 9, (16, 16)).astype(float)
    lanes = np.arange(64)
    a = Am[lanes % 16, lanes // 16]
    b = Bm[lanes // 16, lanes % 16]
    c = np.stack([Cm[lanes // 16 + 4 * v, lanes % 16] for v in range(4)], axis=1)
    d = microbench.mfma_once(a, b, c).numpy()
    D = Am @ Bm + Cm
    want = np.stack([D[lanes // 16 + 4 * v, lanes % 16] for v in range(4)], axis=1)
    assert np.array_equal(d, want)
