"""Pins for the CPU oracle: facts fixed by the GEMM definition (the paper's
Eq. 1, Section II) and by mathematics, not by the oracle's own code.

Each pin is chosen so that a plausible slip in the oracle -- a dropped term,
a wrong sign, a wrong index or leading dimension, a transposed operand, a
mishandled alpha/beta special case -- fails at least one of them.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg.blas as sblas

import oracle
from tests.colmajor import gamma, load, op, rel_frobenius, store


def _run(ta, tb, A, B, C0, alpha, beta, lda=None, ldb=None, ldc=None):
    """Run the oracle on ordinary matrices; returns (result, storage of C)."""
    Am, Bm = np.asarray(A, float), np.asarray(B, float)
    m = op(Am, ta).shape[0]
    k = op(Am, ta).shape[1]
    n = op(Bm, tb).shape[1]
    As, Bs, Cs = store(Am, lda), store(Bm, ldb), store(C0, ldc)
    info = oracle.gemm(ta, tb, m, n, k, alpha, As, As.shape[1], Bs, Bs.shape[1], beta,
                       Cs, Cs.shape[1])
    assert info == 0
    return load(Cs, m), Cs


rng = np.random.default_rng(12345)


# P1 -- identity: I*B = B and A*I = A, exactly (each sum has one nonzero term)
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.0, 1.0), (-0.5, 2.0), (3.0, -1.25)])
def test_identity_left_and_right(ta, tb, alpha, beta):
    m, n = 13, 7
    X = rng.uniform(-1, 1, (m, n))
    C0 = rng.uniform(-1, 1, (m, n))
    # left identity: op(A) = I_m, op(B) = X
    B = X.T if tb == "T" else X
    got, _ = _run(ta, tb, np.eye(m), B, C0, alpha, beta, lda=m + 3, ldb=B.shape[0] + 2, ldc=m + 1)
    assert np.array_equal(got, alpha * X + beta * C0)
    # right identity: op(A) = X, op(B) = I_n
    A = X.T if ta == "T" else X
    got, _ = _run(ta, tb, A, np.eye(n), C0, alpha, beta, lda=A.shape[0] + 5)
    assert np.array_equal(got, alpha * X + beta * C0)


# P2 -- permutation / row selection: (S*B)(r, :) = B(s(r), :), exactly
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
def test_selection_and_permutation(ta, tb):
    m, k, n = 9, 14, 11
    s = rng.permutation(k)[:m]                 # injective row choice
    S = np.zeros((m, k)); S[np.arange(m), s] = 1.0
    Bop = rng.uniform(-1, 1, (k, n))
    A = S.T if ta == "T" else S
    B = Bop.T if tb == "T" else Bop
    got, _ = _run(ta, tb, A, B, np.zeros((m, n)), 1.0, 0.0, lda=A.shape[0] + 1, ldb=B.shape[0] + 4)
    assert np.array_equal(got, Bop[s, :])
    # column permutation from the right: (X * P)(:, j) = X(:, sigma^-1(j))
    sigma = rng.permutation(n)
    P = np.zeros((n, n)); P[np.arange(n), sigma] = 1.0
    X = rng.uniform(-1, 1, (m, n))
    A = X.T if ta == "T" else X
    B = P.T if tb == "T" else P
    got, _ = _run(ta, tb, A, B, np.zeros((m, n)), 1.0, 0.0)
    inv = np.argsort(sigma)
    assert np.array_equal(got, X[:, inv])


# P3 -- rank one: k = 1 has a closed form with a single rounded product
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.75, -1.5), (-2.0, 1.0)])
def test_rank_one_k1(alpha, beta):
    m, n = 17, 5
    a = rng.uniform(-1, 1, (m, 1)); b = rng.uniform(-1, 1, (1, n))
    C0 = rng.uniform(-1, 1, (m, n))
    got, _ = _run("N", "N", a, b, C0, alpha, beta)
    prod = a * b                                     # fl(a_r * b_c)
    exp = alpha * prod + beta * C0 if beta != 0 else alpha * prod
    assert np.array_equal(got, exp)


def test_rank_one_integer_closed_form():
    # A = u v^T, B = w z^T  =>  A B = (v . w) u z^T, all exact in binary64
    m, k, n = 21, 33, 19
    u = rng.integers(-9, 10, m); v = rng.integers(-9, 10, k)
    w = rng.integers(-9, 10, k); z = rng.integers(-9, 10, n)
    A = np.outer(u, v).astype(float); B = np.outer(w, z).astype(float)
    got, _ = _run("N", "N", A, B, np.zeros((m, n)), 1.0, 0.0)
    exp = float(np.dot(v, w)) * np.outer(u, z).astype(float)
    assert np.array_equal(got, exp)


# P4 -- small integers: every partial sum is an exact integer, so any
# summation order gives the exact product; compare with integer arithmetic.
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (7, 9, 8), (16, 15, 17), (33, 31, 64),
                                   (65, 63, 129), (5, 3, 513), (64, 64, 64)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-1.0, 1.0), (2.0, 0.5), (0.5, -2.0),
                                        (0.0, 1.0), (0.0, -1.0)])
def test_small_integers_exact(m, n, k, alpha, beta):
    Ai = rng.integers(-32, 33, (m, k)); Bi = rng.integers(-32, 33, (k, n))
    C0i = rng.integers(-32, 33, (m, n))
    exact = Ai @ Bi                                   # int64, exact
    for ta, tb in [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")]:
        A = Ai.T if ta == "T" else Ai
        B = Bi.T if tb == "T" else Bi
        got, _ = _run(ta, tb, A, B, C0i.astype(float), alpha, beta,
                      lda=A.shape[0] + (k % 3), ldb=B.shape[0] + 1, ldc=m + 2)
        exp = np.array([[Fraction(alpha) * int(exact[r, c]) + Fraction(beta) * int(C0i[r, c])
                         for c in range(n)] for r in range(m)], dtype=object)
        assert np.array_equal(got, exp.astype(float)), (ta, tb)


# P5 -- brute force against exact rational arithmetic, within Higham's bound
def _exact(ta, tb, A, B, C0, alpha, beta):
    Ao, Bo = op(A, ta), op(B, tb)
    m, k = Ao.shape; n = Bo.shape[1]
    out = np.empty((m, n), dtype=object)
    for r in range(m):
        for c in range(n):
            s = sum((Fraction(Ao[r, p]) * Fraction(Bo[p, c]) for p in range(k)), Fraction(0))
            out[r, c] = Fraction(alpha) * s + Fraction(beta) * Fraction(C0[r, c])
    return out


def test_brute_force_tiny_all_shapes():
    checked = 0
    for m, n, k in itertools.product(range(1, 5), repeat=3):
        for ta, tb in itertools.product("NT", "NT"):
            Aop = rng.uniform(-1, 1, (m, k)); Bop = rng.uniform(-1, 1, (k, n))
            A = Aop.T.copy() if ta == "T" else Aop
            B = Bop.T.copy() if tb == "T" else Bop
            C0 = rng.uniform(-1, 1, (m, n))
            for alpha, beta in itertools.product([0.0, 1.0, -1.0, 0.5], repeat=2):
                got, _ = _run(ta, tb, A, B, C0, alpha, beta, lda=A.shape[0] + 1)
                ex = _exact(ta, tb, A, B, C0, alpha, beta)
                bound = gamma(k + 2) * (abs(alpha) * (np.abs(Aop) @ np.abs(Bop)) + abs(beta) * np.abs(C0))
                err = np.array([[abs(Fraction(got[r, c]) - ex[r, c]) for c in range(n)]
                                for r in range(m)], dtype=object)
                assert np.all(err.astype(float) <= bound), (m, n, k, ta, tb, alpha, beta)
                checked += 1
    assert checked == 64 * 4 * 16


# P6 -- independent library implementations (OpenBLAS via numpy and scipy)
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("m,n,k", [(32, 32, 32), (57, 13, 100), (100, 71, 9)])
def test_against_blas(ta, tb, m, n, k):
    Aop = rng.uniform(-1, 1, (m, k)); Bop = rng.uniform(-1, 1, (k, n))
    C0 = rng.uniform(-1, 1, (m, n))
    A = Aop.T.copy() if ta == "T" else Aop
    B = Bop.T.copy() if tb == "T" else Bop
    got, _ = _run(ta, tb, A, B, C0, 0.7, -0.3)
    ref_np = 0.7 * (Aop @ Bop) - 0.3 * C0
    ref_sp = sblas.dgemm(0.7, A, B, beta=-0.3, c=C0.copy(order="F"),
                         trans_a=(ta == "T"), trans_b=(tb == "T"))
    assert rel_frobenius(got, ref_np) <= 1e-14
    assert rel_frobenius(got, ref_sp) <= 1e-14


# P7 -- spectral structure: A = Q Da Q^T, B = Q Db Q^T  =>  AB = Q Da Db Q^T
def test_spectral_same_basis():
    from paper_2203_09353_amd.inputs import haar_orthogonal
    size = 48
    Q = haar_orthogonal(7, 0, 1, size)[0].numpy()
    da = rng.uniform(-1, 1, size); db = rng.uniform(-1, 1, size)
    A = (Q * da) @ Q.T; B = (Q * db) @ Q.T
    C0 = rng.uniform(-1, 1, (size, size))
    got, _ = _run("N", "N", A, B, C0, 1.0, 1.0)
    assert abs(np.trace(got) - (np.sum(da * db) + np.trace(C0))) <= 1e-12
    got0, _ = _run("N", "N", A, B, np.zeros((size, size)), 1.0, 0.0)
    assert abs(np.linalg.norm(got0) ** 2 - np.sum((da * db) ** 2)) <= 1e-12
    assert rel_frobenius(got0, (Q * (da * db)) @ Q.T) <= 1e-13


def test_spectral_symmetric_swap():
    # for symmetric A, B with different bases: (AB)^T = B A
    from paper_2203_09353_amd.inputs import haar_orthogonal
    size = 40
    Qs = haar_orthogonal(8, 0, 2, size).numpy()
    A = (Qs[0] * rng.uniform(-1, 1, size)) @ Qs[0].T
    B = (Qs[1] * rng.uniform(-1, 1, size)) @ Qs[1].T
    A = 0.5 * (A + A.T); B = 0.5 * (B + B.T)
    ab, _ = _run("N", "N", A, B, np.zeros((size, size)), 1.0, 0.0)
    ba, _ = _run("N", "N", B, A, np.zeros((size, size)), 1.0, 0.0)
    assert rel_frobenius(ab.T, ba) <= 1e-13
    # and the transposed-operand route gives the same product: A^T B^T = (BA)^T... = AB
    abt, _ = _run("T", "T", A, B, np.zeros((size, size)), 1.0, 0.0)
    assert rel_frobenius(abt, ba.T) <= 1e-13


# P8 -- linearity in alpha and beta (power-of-two scalars, integer data: exact)
def test_linearity_alpha_beta():
    m, n, k = 23, 19, 40
    A = rng.integers(-32, 33, (m, k)).astype(float)
    B = rng.integers(-32, 33, (k, n)).astype(float)
    C0 = rng.integers(-32, 33, (m, n)).astype(float)
    g10, _ = _run("N", "N", A, B, C0, 1.0, 0.0)
    for alpha, beta in [(2.0, 1.0), (-4.0, 0.5), (0.25, -2.0), (1.0, 1.0)]:
        g, _ = _run("N", "N", A, B, C0, alpha, beta)
        assert np.array_equal(g, alpha * g10 + beta * C0)


# P9 -- canaries: padding is never read or written; beta == 0 never reads C;
# alpha == 0 never reads A or B
def test_padding_and_special_case_canaries():
    m, n, k = 10, 6, 7
    A = rng.uniform(-1, 1, (m, k)); B = rng.uniform(-1, 1, (k, n))
    C0 = np.full((m, n), np.nan)
    As, Bs, Cs = store(A, m + 5), store(B, k + 3), store(C0, m + 4)
    Cs[:, m:] = -7.25                                # padding sentinel in C
    assert oracle.gemm("N", "N", m, n, k, 1.0, As, m + 5, Bs, k + 3, 0.0, Cs, m + 4) == 0
    assert not np.isnan(Cs[:, :m]).any()
    assert np.all(Cs[:, m:] == -7.25)
    assert rel_frobenius(load(Cs, m), A @ B) <= 1e-14
    # alpha == 0: A and B are NaN and must not be read
    An, Bn = store(np.full((m, k), np.nan)), store(np.full((k, n), np.nan))
    C1 = rng.uniform(-1, 1, (m, n)); Cs1 = store(C1)
    assert oracle.gemm("N", "N", m, n, k, 0.0, An, m, Bn, k, -3.0, Cs1, m) == 0
    assert np.array_equal(load(Cs1, m), -3.0 * C1)
    # alpha == 0 and beta == 0: C becomes exactly zero even from NaN
    Cs2 = store(np.full((m, n), np.nan))
    assert oracle.gemm("N", "N", m, n, k, 0.0, An, m, Bn, k, 0.0, Cs2, m) == 0
    assert np.all(load(Cs2, m) == 0.0)


# P10 -- degenerate sizes
def test_degenerate_sizes():
    C0 = rng.uniform(-1, 1, (5, 4))
    Cs = store(C0)
    # k == 0: C = beta C
    assert oracle.gemm("N", "N", 5, 4, 0, 1.0, np.zeros(1), 5, np.zeros(1), 1, 0.5, Cs, 5) == 0
    assert np.array_equal(load(Cs, 5), 0.5 * C0)
    # k == 0, beta == 1: untouched (bit-identical, negative zero included)
    Cs[1, 2] = -0.0
    before = Cs.copy()
    assert oracle.gemm("N", "N", 5, 4, 0, 2.0, np.zeros(1), 5, np.zeros(1), 1, 1.0, Cs, 5) == 0
    assert np.array_equal(before.view(np.int64), Cs.view(np.int64))
    # m == 0 or n == 0: nothing happens
    assert oracle.gemm("N", "N", 0, 4, 3, 1.0, np.zeros(1), 1, np.zeros(12), 3, 0.0, Cs, 1) == 0
    assert oracle.gemm("N", "N", 5, 0, 3, 1.0, np.zeros(15), 5, np.zeros(1), 3, 0.0, Cs, 5) == 0
    assert np.array_equal(before, Cs)
    # empty batch
    oracle.gemm_batched("N", "N", 3, 3, 3, 1.0, [], [], 0.0, [])


def test_argument_rules_order():
    # reference-BLAS argument numbers: first failing rule wins
    assert oracle.check_args("X", "N", 1, 1, 1, 1, 1, 1) == -1
    assert oracle.check_args("N", "?", 1, 1, 1, 1, 1, 1) == -2
    assert oracle.check_args("N", "N", -1, 1, 1, 1, 1, 1) == -3
    assert oracle.check_args("N", "N", 1, -1, 1, 1, 1, 1) == -4
    assert oracle.check_args("N", "N", 1, 1, -1, 1, 1, 1) == -5
    assert oracle.check_args("N", "N", 4, 1, 2, 3, 2, 4) == -8       # lda < m
    assert oracle.check_args("T", "N", 4, 1, 2, 1, 2, 4) == -8       # lda < k for 'T'
    assert oracle.check_args("N", "N", 4, 3, 2, 4, 1, 4) == -10      # ldb < k
    assert oracle.check_args("N", "T", 4, 3, 2, 4, 2, 4) == -10      # ldb < n for 'T'
    assert oracle.check_args("N", "N", 4, 3, 2, 4, 2, 3) == -13      # ldc < m
    assert oracle.check_args("n", "c", 0, 0, 0, 1, 1, 1) == 0        # lower case, zero sizes
    assert oracle.check_args("N", "N", 0, 0, 0, 0, 1, 1) == -8       # ld >= 1 always


def test_batched_threads_deterministic_and_independent():
    batch, m, n, k = 40, 24, 17, 31
    A = rng.uniform(-1, 1, (batch, k, m)); B = rng.uniform(-1, 1, (batch, n, k))
    C0 = rng.uniform(-1, 1, (batch, n, m))
    C1, C8 = C0.copy(), C0.copy()
    oracle.gemm_batched("N", "N", m, n, k, 1.5, A, B, 0.5, C1, nthreads=1)
    oracle.gemm_batched("N", "N", m, n, k, 1.5, A, B, 0.5, C8, nthreads=8)
    assert np.array_equal(C1, C8)
    # each instance equals the single-instance call
    for i in (0, 17, 39):
        Ci = C0[i].copy()
        oracle.gemm("N", "N", m, n, k, 1.5, A[i], m, B[i], k, 0.5, Ci, m)
        assert np.array_equal(Ci, C1[i])


def test_vbatched_info_and_skip():
    ms = [3, -1, 4, 5]; ns = [2, 2, 3, 1]; ks = [4, 4, 0, 2]
    As = [rng.uniform(-1, 1, (max(k, 1), max(m, 1))) for m, k in zip(ms, ks)]
    Bs = [rng.uniform(-1, 1, (n, max(k, 1))) for n, k in zip(ns, ks)]
    Cs = [rng.uniform(-1, 1, (n, max(m, 1))) for m, n in zip(ms, ns)]
    Cs[3] = rng.uniform(-1, 1, (1, 4))                # ldc = 4 < m = 5: invalid
    C_before = [c.copy() for c in Cs]
    info = oracle.gemm_vbatched("N", "N", ms, ns, ks, 1.0, As, Bs, 0.5, Cs)
    assert list(info) == [0, -3, 0, -13]
    assert np.array_equal(Cs[1], C_before[1]) and np.array_equal(Cs[3], C_before[3])
    assert np.array_equal(Cs[2], 0.5 * C_before[2])                  # k == 0
    ref = load(As[0], 3) @ load(Bs[0], 4) + 0.5 * load(C_before[0], 3)
    assert rel_frobenius(load(Cs[0], 3), ref) <= 1e-14
