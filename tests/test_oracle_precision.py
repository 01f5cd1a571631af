"""Pins for the precision-mode oracle (oracle/precision.py): exact digit
reconstruction, bfloat16 rounding against torch's conversion, exactness on
integer data, an error bound derived from the dropped slice terms checked
against exact rational arithmetic, and convergence with the slice count."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import precision as P

rng = np.random.default_rng(77)


@pytest.mark.parametrize("s", range(1, 9))
def test_digits_reconstruct_exactly(s):
    x = np.concatenate([rng.uniform(-1, 1, 400), [0.0, 0.5, -0.5, 2.0 ** -30, -0.999999999999,
                                                  1 / 256 + 1 / 512, -(1 / 128) * 0.5]])
    d, r = P.digits(x, s)
    for t in range(s):
        assert np.all(np.abs(d[t]) <= 128)
    assert np.all(np.abs(r) <= 0.5)
    for idx in range(len(x)):
        tot = sum(Fraction(int(d[t][idx])) * Fraction(2) ** (-7 - 8 * t) for t in range(s))
        tot += Fraction(float(r[idx])) * Fraction(2) ** (-7 - 8 * (s - 1))
        assert tot == Fraction(float(x[idx]))


def test_bf16_rounding_matches_torch():
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9]])
    ours = P.round_bf16(x)
    ref = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    assert np.array_equal(ours, ref.numpy())


@pytest.mark.parametrize("s", [1, 2, 3, 6])
def test_integer_data_is_exact(s):
    # integers below 2^7 in magnitude are single digits after chunk scaling
    m, k, n = 9, 70, 11
    A = rng.integers(-127, 128, (m, k)).astype(float)
    B = rng.integers(-127, 128, (k, n)).astype(float)
    C = P.emulated_gemm(A, B, s)
    assert np.array_equal(C, (A.astype(np.int64) @ B.astype(np.int64)).astype(float))


def _bound(A, B, s):
    """|emu_s - AB| <= per chunk 2^(e+f) (len (s+2) 2^-8s) + rounding of the
    recombination, see the module docstring: dropped slice pairs (g > s+1)
    contribute at most (s - 1) 2^-8s per scaled product, the two remainders
    2^-8s each and their product less; each of the s + chunks rounded adds
    contributes at most u times the magnitude it works on."""
    m, k = A.shape
    n = B.shape[1]
    u = 2.0 ** -53
    trunc = np.zeros((m, n))
    mag = np.zeros((m, n))
    for c0 in range(0, k, P.CHUNK):
        c1 = min(k, c0 + P.CHUNK)
        e = P.chunk_exponents_rows(A, c0, c1)
        f = P.chunk_exponents_rows(B.T, c0, c1)
        sc = np.ldexp(np.ones((m, n)), e[:, None] + f[None, :])
        trunc += sc * (c1 - c0) * (s + 2) * 2.0 ** (-8 * s)
        mag += np.abs(A[:, c0:c1]) @ np.abs(B[c0:c1, :])
    nchunks = (k + P.CHUNK - 1) // P.CHUNK
    return trunc + 2 * (s + nchunks + 2) * u * (mag + trunc)


@pytest.mark.parametrize("s", [1, 2, 3, 4, 6, 7, 8])
def test_error_within_derived_bound(s):
    m, k, n = 4, 45, 3
    A = rng.uniform(-1, 1, (m, k)) * 2.0 ** rng.integers(-20, 21, (m, k))
    B = rng.uniform(-1, 1, (k, n)) * 2.0 ** rng.integers(-20, 21, (k, n))
    C = P.emulated_gemm(A, B, s)
    bound = _bound(A, B, s)
    for i in range(m):
        for j in range(n):
            exact = sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(k))
            assert abs(Fraction(float(C[i, j])) - exact) <= Fraction(float(bound[i, j])), (s, i, j)


def test_error_falls_with_slices():
    m, k, n = 16, 256, 16
    A = rng.uniform(1, 2, (m, k)) * rng.choice([-1, 1], (m, k)) * 2.0 ** rng.integers(-20, 21, (m, k))
    B = rng.uniform(1, 2, (k, n)) * rng.choice([-1, 1], (k, n)) * 2.0 ** rng.integers(-20, 21, (k, n))
    exact = A @ B   # binary64 reference; far below the slice truncation for s <= 5
    errs = [P.relative_errors(P.emulated_gemm(A, B, s), exact)[0] for s in range(1, 6)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 32
    assert errs[0] < 0.05


def test_alpha_beta_follow_the_binary64_rules():
    A = rng.uniform(-1, 1, (5, 40)); B = rng.uniform(-1, 1, (40, 6)); C0 = rng.uniform(-1, 1, (5, 6))
    acc = P.emulated_gemm(A, B, 4)
    assert np.array_equal(P.emulated_gemm(A, B, 4, 2.0, 0.5, C0), 2.0 * acc + 0.5 * C0)
    assert np.array_equal(P.emulated_gemm(A, B, 4, 1.0, 0.0, np.full((5, 6), np.nan)), acc)


def test_reference_products_of_rounded_inputs():
    A = rng.standard_normal((7, 33)); B = rng.standard_normal((33, 5))
    r32 = P.reference_product(A, B, "fp32")
    assert np.array_equal(r32, A.astype(np.float32).astype(np.float64) @
                          B.astype(np.float32).astype(np.float64))
    rb = P.reference_product(A, B, "bf16")
    ta = torch.tensor(A).float().bfloat16().double().numpy()
    tb = torch.tensor(B).float().bfloat16().double().numpy()
    assert np.array_equal(rb, ta @ tb)


def test_dot2_against_exact_rationals():
    # Ogita-Rump-Oishi bound: |res - exact| <= u |exact| + gamma_k^2 (|A||B|)
    u = 2.0 ** -53
    for trial in range(4):
        m, k, n = 3, 37, 4
        A = rng.uniform(-1, 1, (m, k)) * 2.0 ** rng.integers(-30, 31, (m, k))
        B = rng.uniform(-1, 1, (k, n)) * 2.0 ** rng.integers(-30, 31, (k, n))
        R = P.dot2_gemm(A, B)
        g = k * u / (1 - k * u)
        mag = np.abs(A) @ np.abs(B)
        for i in range(m):
            for j in range(n):
                exact = sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(k))
                err = abs(Fraction(float(R[i, j])) - exact)
                assert err <= Fraction(u) * abs(exact) + Fraction(g * g * float(mag[i, j]))


def test_dot2_cancellation_beyond_binary64():
    # exact result 1; a plain binary64 sum in this order returns 0
    A = np.array([[1e16, 1.0, -1e16]])
    B = np.ones((3, 1))
    assert (1e16 + 1.0) - 1e16 == 0.0
    assert P.dot2_gemm(A, B)[0, 0] == 1.0
    # error-free transformations are exact
    a, b = 0.1, 3.0 ** -20
    s, e = P._two_sum(a, b)
    assert Fraction(s) + Fraction(e) == Fraction(a) + Fraction(b)
    p, e = P._two_product(a, b)
    assert Fraction(p) + Fraction(e) == Fraction(a) * Fraction(b)


# ---- i8emu<s>: whole-row scaling, signed int8 digits, exact integer diagonals

@pytest.mark.parametrize("s", range(1, 9))
def test_int8_digits_reconstruct_exactly(s):
    lim = 2 ** (8 * s - 2)
    X = np.concatenate([rng.integers(-lim, lim + 1, 500, dtype=np.int64),
                        np.array([0, 1, -1, 127, 128, -128, -129, 255, 256, lim, -lim, lim - 1,
                                  -lim + 1, lim // 2, -(lim // 2) - 128], dtype=np.int64)])
    X = np.clip(X, -lim, lim)
    d = P.int8_digits(X, s)
    assert np.all(np.abs(d[0]) <= 64)
    for t in range(1, s):
        assert np.all((d[t] >= -128) & (d[t] <= 127))
    for idx in range(len(X)):
        tot = sum(int(d[t][idx]) * 256 ** (s - 1 - t) for t in range(s))
        assert tot == int(X[idx])


@pytest.mark.parametrize("s", [3, 4, 6, 7, 8])
def test_int8_integer_data_is_exact(s):
    # integers of at most 8 bits scale to X with >= 8s - 10 trailing zero
    # bits: only the top two digits are non-zero, all their pairs are kept
    m, k, n = 9, 70, 11
    A = rng.integers(-255, 256, (m, k)).astype(float)
    B = rng.integers(-255, 256, (k, n)).astype(float)
    A[3, :] = 0.0
    B[:, 4] = rng.integers(-3, 4, k)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(float)
    assert np.array_equal(P.int8_emulated_gemm(A, B, s), exact)
    C0 = rng.integers(-50, 50, (m, n)).astype(float)
    assert np.array_equal(P.int8_emulated_gemm(A, B, s, -2.0, 0.5, C0), -2.0 * exact + 0.5 * C0)


def _bound8(A, B, s):
    """Step 2 rounds each scaled entry by at most 1/2 (2^(2-8s) relative to
    the row scale), the dropped pairs of step 4 add at most
    1.004 (s - 1) 2^(2-8s) per product, so k products give
    1.02 s k 2^(2-8s) 2^(e+f); step 5's s - 1 rounded adds work on at most
    1.02 k 2^(e+f) each, and the sum itself is rounded once more."""
    m, k = A.shape
    n = B.shape[1]
    u = 2.0 ** -53
    e = P.row_exponents(A)
    f = P.row_exponents(B.T)
    sc = np.ldexp(np.ones((m, n)), e[:, None] + f[None, :]) * k
    return 1.02 * s * 2.0 ** (2 - 8 * s) * sc + 1.05 * s * u * sc + 2 * u * (np.abs(A) @ np.abs(B))


@pytest.mark.parametrize("s", [1, 2, 3, 5, 6, 7, 8])
@pytest.mark.parametrize("spread", [20, 300])
def test_int8_error_within_derived_bound(s, spread):
    m, k, n = 4, 45, 3
    A = rng.uniform(-1, 1, (m, k)) * 2.0 ** rng.integers(-spread, spread + 1, (m, k))
    B = rng.uniform(-1, 1, (k, n)) * 2.0 ** rng.integers(-spread, spread + 1, (k, n))
    C = P.int8_emulated_gemm(A, B, s)
    bound = _bound8(A, B, s)
    for i in range(m):
        for j in range(n):
            exact = sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(k))
            assert abs(Fraction(float(C[i, j])) - exact) <= Fraction(float(bound[i, j])), (s, i, j)


def test_int8_error_falls_with_slices_and_reaches_binary64():
    m, k, n = 16, 256, 16
    A = rng.uniform(1, 2, (m, k)) * rng.choice([-1, 1], (m, k)) * 2.0 ** rng.integers(-20, 21, (m, k))
    B = rng.uniform(1, 2, (k, n)) * rng.choice([-1, 1], (k, n)) * 2.0 ** rng.integers(-20, 21, (k, n))
    ref = P.dot2_gemm(A, B)
    errs = [P.relative_errors(P.int8_emulated_gemm(A, B, s), ref)[0] for s in range(1, 9)]
    for a, b in zip(errs[:6], errs[1:7]):
        assert b < a / 64
    # whole-row scaling costs the bits between an entry and its row's
    # largest: on 2^+-20 data seven slices stay within 1e-14, eight are as
    # accurate as the binary64 product itself
    assert errs[6] < 1e-14
    assert errs[7] <= P.relative_errors(A @ B, ref)[0]


def test_int8_single_term_and_zero_rows():
    # k = 1 is a rank-one outer product: with s >= 7 (54 digit bits, more
    # than binary64's 53) every product of two doubles is reproduced to the
    # last bit when the product is exact in binary64
    a = np.array([[1.5], [-0.75], [0.0], [3.0 * 2.0 ** 40]])
    b = np.array([[2.0, -1.25, 2.0 ** -30]])
    for s in (7, 8):
        assert np.array_equal(P.int8_emulated_gemm(a, b, s), a @ b)
    Z = np.zeros((3, 5))
    assert np.array_equal(P.int8_emulated_gemm(Z, rng.uniform(-1, 1, (5, 2)), 4), np.zeros((3, 2)))


@pytest.mark.parametrize("s", [1])
def test_int8_rank_one_error_is_rounding_not_truncation(s):
    # k = 1 and one slice: no pair is dropped, the only error is the scaling
    # to integers (step 2); rounding to nearest keeps it within
    # 2^(e+f) (2^(2-8s) + 2^(4-16s)) of the exact product for every entry
    # (truncation would reach twice that)
    a = rng.uniform(-1, 1, (60, 1)) * 2.0 ** rng.integers(-5, 6, (60, 1))
    b = rng.uniform(-1, 1, (1, 60)) * 2.0 ** rng.integers(-5, 6, (1, 60))
    C = P.int8_emulated_gemm(a, b, s)
    e = P.row_exponents(a)
    f = P.row_exponents(b.T)
    lim = Fraction(2) ** (2 - 8 * s) + Fraction(2) ** (4 - 16 * s)
    worst = Fraction(0)
    for i in range(60):
        for j in range(60):
            err = abs(Fraction(float(C[i, j])) - Fraction(float(a[i, 0])) * Fraction(float(b[0, j])))
            rel = err / Fraction(2) ** int(e[i] + f[j])
            assert rel <= lim, (i, j)
            worst = max(worst, rel)
    assert worst > lim / 4          # the bound is nearly reached: the test is sharp
