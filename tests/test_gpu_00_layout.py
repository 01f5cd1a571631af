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


def test_mfma_4x4x4_lane_layout():
    """Pins the layout of v_mfma_f64_4x4x4_4b_f64 the tile kernels use: for
    block b, lane 16 s + 4 b + i holds A_b(i, s), lane 16 s + 4 b + j holds
    B_b(s, j), and D_b(i, j) (and C_b(i, j)) live in lane 16 i + 4 b + j."""
    from paper_2203_09353_amd import microbench
    rng = np.random.default_rng(1)
    A = rng.integers(-8, 9, (4, 4, 4)).astype(float)   # [b, i, s]
    B = rng.integers(-8, 9, (4, 4, 4)).astype(float)   # [b, s, j]
    C = rng.integers(-8, 9, (4, 4, 4)).astype(float)   # [b, i, j]
    a = np.zeros(64); b = np.zeros(64); c = np.zeros(64)
    for blk in range(4):
        for x in range(4):
            for y in range(4):
                a[16 * y + 4 * blk + x] = A[blk, x, y]
                b[16 * x + 4 * blk + y] = B[blk, x, y]
                c[16 * x + 4 * blk + y] = C[blk, x, y]
    d = microbench.mfma4_once(a, b, c).numpy()
    D = A @ B + C
    want = np.zeros(64)
    for blk in range(4):
        for i in range(4):
            for j in range(4):
                want[16 * i + 4 * blk + j] = D[blk, i, j]
    assert np.array_equal(d, want)


def test_mfma_f32_16x16x4_lane_layout():
    """v_mfma_f32_16x16x4_f32 (precision mode fp32): lane l holds A(l%16, l/16)
    and B(l/16, l%16); result register v of lane l is D(4 (l/16) + v, l%16)."""
    from paper_2203_09353_amd import microbench
    rng = np.random.default_rng(2)
    Am = rng.integers(-8, 9, (16, 4)).astype(np.float32)
    Bm = rng.integers(-8, 9, (4, 16)).astype(np.float32)
    Cm = rng.integers(-8, 9, (16, 16)).astype(np.float32)
    lanes = np.arange(64)
    a = Am[lanes % 16, lanes // 16]
    b = Bm[lanes // 16, lanes % 16]
    c = np.stack([Cm[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    d = microbench.mfma_f32_once(a, b, c).numpy()
    D = Am @ Bm + Cm
    want = np.stack([D[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    assert np.array_equal(d, want)


def test_mfma_bf16_16x16x32_lane_layout():
    """v_mfma_f32_16x16x32_bf16 (precision modes bf16 and emulated): lane l
    holds A(l%16, 8 (l/16) + e) and B(8 (l/16) + e, l%16), e = 0..7; result
    register v of lane l is D(4 (l/16) + v, l%16)."""
    from paper_2203_09353_amd import microbench
    rng = np.random.default_rng(3)
    Am = rng.integers(-8, 9, (16, 32)).astype(np.float32)
    Bm = rng.integers(-8, 9, (32, 16)).astype(np.float32)
    Cm = rng.integers(-8, 9, (16, 16)).astype(np.float32)
    lanes = np.arange(64)
    a = np.stack([Am[lanes % 16, 8 * (lanes // 16) + e] for e in range(8)], axis=1)
    b = np.stack([Bm[8 * (lanes // 16) + e, lanes % 16] for e in range(8)], axis=1)
    c = np.stack([Cm[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    d = microbench.mfma_bf16_once(a, b, c).numpy()
    D = Am @ Bm + Cm
    want = np.stack([D[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    assert np.array_equal(d, want)


def test_mfma_i8_16x16x64_lane_layout():
    """v_mfma_i32_16x16x64_i8 (emulated mode on int8 digits): lane l holds
    A(l%16, 16 (l/16) + e) and B(16 (l/16) + e, l%16) in byte e = 0..15 of
    its 16-byte operand; result register v of lane l is D(4 (l/16) + v, l%16).
    Extreme digits (-128, 127) included: products and sums are exact int32."""
    from paper_2203_09353_amd import microbench
    rng = np.random.default_rng(4)
    Am = rng.integers(-128, 128, (16, 64))
    Bm = rng.integers(-128, 128, (64, 16))
    Am[0, :] = -128
    Bm[:, 0] = -128
    Am[1, :] = 127
    Cm = rng.integers(-2 ** 20, 2 ** 20, (16, 16))
    lanes = np.arange(64)
    a = np.stack([Am[lanes % 16, 16 * (lanes // 16) + e] for e in range(16)], axis=1)
    b = np.stack([Bm[16 * (lanes // 16) + e, lanes % 16] for e in range(16)], axis=1)
    c = np.stack([Cm[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    d = microbench.mfma_i8_once(a, b, c).numpy()
    D = Am @ Bm + Cm
    want = np.stack([D[4 * (lanes // 16) + v, lanes % 16] for v in range(4)], axis=1)
    assert np.array_equal(d, want)
