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
