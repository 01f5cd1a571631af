"""The pins of the int8-digit emulated mode have teeth: plant plausible
mistakes in a copy of the oracle's functions (on the CPU, from their source
text), and check that the pin checks below reject every mutant while
accepting the unmodified functions."""
import inspect
from fractions import Fraction

import numpy as np
import pytest

from oracle import precision as P

SRC = "\n".join(inspect.getsource(f) for f in (P.row_exponents, P.int8_digits,
                                                P.int8_emulated_gemm))

# (name, original text, mutated text)
MUTANTS = [
    ("dropped_top_diagonal", "for g in range(2, s + 2):", "for g in range(2, s + 1):"),
    ("wrong_final_shift", "- 12)", "- 11)"),
    ("wrong_diagonal_weight", "T * 2.0 ** -8", "T * 2.0 ** -7"),
    ("wrong_digit_offset", "np.mod(X + 128, 256) - 128", "np.mod(X + 127, 256) - 127"),
    ("column_exponents_from_rows", "f = row_exponents(B.T)", "f = row_exponents(B)"),
    ("one_bit_less_scaling", "(8 * s - 2) - e[:, None]", "(8 * s - 3) - e[:, None]"),
    ("truncation_not_rounding", "X = np.rint(np.ldexp(A", "X = np.trunc(np.ldexp(A"),
    ("reversed_digit_order", "[X] + low[::-1]", "[X] + low"),
    ("max_not_abs", "np.max(np.abs(A), axis=1)", "np.max(A, axis=1)"),
]


def _build(src):
    ns = {"np": np}
    exec(src, ns)
    return ns["int8_digits"], ns["int8_emulated_gemm"], ns["row_exponents"]


def _pins_pass(digits, gemm, rowexp):
    """True when every pin below holds (a compact replay of the pins in
    test_oracle_precision.py)."""
    return _first_failure(digits, gemm, rowexp) is None


def _first_failure(digits, gemm, rowexp):
    """Name of the first pin that fails, None if all hold."""
    rng = np.random.default_rng(5)
    try:
        # digit reconstruction and ranges
        for s in (1, 3, 7):
            lim = 2 ** (8 * s - 2)
            X = np.concatenate([rng.integers(-lim, lim + 1, 200, dtype=np.int64),
                                np.array([lim, -lim, 127, 128, -129], dtype=np.int64)])
            X = np.clip(X, -lim, lim)
            d = digits(X, s)
            if np.any(np.abs(d[0]) > 64):
                return "digit_top_range"
            if any(np.any((d[t] < -128) | (d[t] > 127)) for t in range(1, s)):
                return "digit_range"
            for i in range(len(X)):
                if sum(int(d[t][i]) * 256 ** (s - 1 - t) for t in range(s)) != int(X[i]):
                    return "digit_reconstruction"
        # exactness on integer data
        A = rng.integers(-255, 256, (7, 40)).astype(float)
        B = rng.integers(-255, 256, (40, 6)).astype(float)
        exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(float)
        if not np.array_equal(gemm(A, B, 4), exact):
            return "integer_exactness"
        # derived bound against exact rationals, wide exponents
        for s in (2, 6):
            A = rng.uniform(-1, 1, (3, 30)) * 2.0 ** rng.integers(-20, 21, (3, 30))
            B = rng.uniform(-1, 1, (30, 3)) * 2.0 ** rng.integers(-20, 21, (30, 3))
            C = gemm(A, B, s)
            e, f = P.row_exponents(A), P.row_exponents(B.T)
            u = 2.0 ** -53
            sc = np.ldexp(np.ones((3, 3)), e[:, None] + f[None, :]) * 30
            bound = (1.02 * s * 2.0 ** (2 - 8 * s) + 1.05 * s * u) * sc + 2 * u * (np.abs(A) @ np.abs(B))
            for i in range(3):
                for j in range(3):
                    ex = sum(Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(30))
                    if abs(Fraction(float(C[i, j])) - ex) > Fraction(float(bound[i, j])):
                        return "derived_bound"
        # rank one, one slice: rounding, not truncation
        a = rng.uniform(-1, 1, (40, 1))
        b = rng.uniform(-1, 1, (1, 40))
        C = gemm(a, b, 1)
        e, f = P.row_exponents(a), P.row_exponents(b.T)
        lim = Fraction(2) ** -6 + Fraction(2) ** -12
        for i in range(40):
            for j in range(40):
                err = abs(Fraction(float(C[i, j])) - Fraction(float(a[i, 0])) * Fraction(float(b[0, j])))
                if err / Fraction(2) ** int(e[i] + f[j]) > lim:
                    return "rank_one_rounding"
        # negative-dominated rows: the exponent follows the magnitude
        A = -np.abs(rng.uniform(0.5, 1, (4, 16))) * 8.0
        B = rng.uniform(-1, 1, (16, 4))
        if np.linalg.norm(gemm(A, B, 7) - A @ B) > 1e-14 * np.linalg.norm(A @ B):
            return "negative_rows"
    except Exception as e:      # a mutant that breaks the computation is caught too
        return "exception: %r" % (e,)
    return None


def test_unmodified_oracle_passes_the_pins():
    assert _first_failure(P.int8_digits, P.int8_emulated_gemm, P.row_exponents) is None
    assert _first_failure(*_build(SRC)) is None


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, orig, mut):
    assert SRC.count(orig) == 1, name
    assert not _pins_pass(*_build(SRC.replace(orig, mut))), name
