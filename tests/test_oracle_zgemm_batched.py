"""Pins for the batched complex oracle (oracle_zgemm_batched in oracle/oracle.c
and its wrapper oracle.zgemm_batched), which the complex GPU tests and the
Gram-product benchmark legs use as their checker.

What fixes the result independently of the oracle: exact Gaussian-integer
arithmetic in Python integers (every instance, every op pair, padded leading
dimensions, NaN canaries in the padding), numpy's complex matmul on random
data, and the definition of a batch (each instance is the single-instance
product of its own operands, whatever the thread count or the order of the
pointer arrays).  Planted mistakes in the batched routine (an instance reading
another instance's operand, swapped leading dimensions, a dropped last
instance, beta taken as alpha) must each fail these pins."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
OPS = [(a, b) for a in "NTC" for b in "NTC"]


def _stored(Xop, t):
    """The stored matrix whose op(.) under `t` is Xop."""
    return Xop if t == "N" else (Xop.T if t == "T" else Xop.conj().T)


def _slab(mats, ld):
    """List of (rows, cols) complex matrices -> (batch, cols, ld) column-major
    storage with NaN in the ld padding."""
    cols = mats[0].shape[1]
    S = np.full((len(mats), cols, ld), complex(np.nan, np.nan))
    for i, X in enumerate(mats):
        S[i, :, :X.shape[0]] = X.T
    return S


def _gauss(rng, shape):
    return (rng.integers(-16, 17, shape) + 1j * rng.integers(-16, 17, shape)).astype(complex)


def _exact(Aop, Bop, alpha, beta, C0):
    """alpha op(A) op(B) + beta C0 in Python integers (Gaussian-integer data)."""
    m, k = Aop.shape
    n = Bop.shape[1]
    out = np.zeros((m, n), complex)
    ar, ai = int(alpha.real), int(alpha.imag)
    br, bi = int(beta.real), int(beta.imag)
    for i in range(m):
        for j in range(n):
            sr = si = 0
            for p in range(k):
                a, b = Aop[i, p], Bop[p, j]
                sr += int(a.real) * int(b.real) - int(a.imag) * int(b.imag)
                si += int(a.real) * int(b.imag) + int(a.imag) * int(b.real)
            cr, ci = int(C0[i, j].real), int(C0[i, j].imag)
            out[i, j] = complex(ar * sr - ai * si + br * cr - bi * ci,
                                ar * si + ai * sr + br * ci + bi * cr)
    return out


def _call_batched(lib, ta, tb, m, n, k, alpha, A, B, beta, C, nthreads=0):
    """oracle_zgemm_batched of `lib` on (batch, cols, ld) slabs (C in place)."""
    pair = lambda z: (ctypes.c_double * 2)(complex(z).real, complex(z).imag)
    arr = lambda S: (ctypes.c_void_p * S.shape[0])(*[S[i].ctypes.data for i in range(S.shape[0])])
    return lib.oracle_zgemm_batched(ta.encode(), tb.encode(), m, n, k, pair(alpha), arr(A),
                                    A.shape[-1], arr(B), B.shape[-1], pair(beta), arr(C),
                                    C.shape[-1], C.shape[0], nthreads)


def _load(so):
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.oracle_zgemm_batched.restype = ctypes.c_int
    L.oracle_zgemm_batched.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, dp, pp, ctypes.c_int, pp, ctypes.c_int, dp,
                                       pp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    return L


def _zb_pins_pass(lib):
    """Gaussian-integer batches, every op pair, distinct padded leading
    dimensions for A, B and C: every instance must equal the exact result,
    padding must keep its NaN, and beta == 0 must not read C."""
    rng = np.random.default_rng(41)
    batch, m, n, k = 5, 6, 4, 7
    for ta, tb in OPS:
        Aops = [_gauss(rng, (m, k)) for _ in range(batch)]
        Bops = [_gauss(rng, (k, n)) for _ in range(batch)]
        C0s = [_gauss(rng, (m, n)) for _ in range(batch)]
        As = [_stored(X, ta) for X in Aops]
        Bs = [_stored(X, tb) for X in Bops]
        A = _slab(As, As[0].shape[0] + 2)
        B = _slab(Bs, Bs[0].shape[0] + 3)
        for alpha, beta in ((1 + 0j, 0j), (2 - 1j, 1 + 3j)):
            C = _slab(C0s, m + 1)
            if beta == 0:
                C[:, :, :m] = complex(np.nan, np.nan)
            if _call_batched(lib, ta, tb, m, n, k, alpha, A, B, beta, C) != 0:
                return False
            for i in range(batch):
                exp = _exact(Aops[i], Bops[i], alpha, beta,
                             C0s[i] if beta != 0 else np.zeros((m, n)))
                if not np.array_equal(C[i, :, :m].T, exp):
                    return False
            if not np.isnan(C[:, :, m:].real).all():
                return False
    return True


def test_batched_gaussian_integers_exact():
    assert _zb_pins_pass(oracle.lib())


@pytest.mark.parametrize("ta,tb", [("N", "N"), ("N", "C"), ("T", "N"), ("C", "T")])
def test_batched_against_numpy(ta, tb):
    rng = np.random.default_rng(43)
    batch, m, n, k = 9, 11, 8, 19
    cplx = lambda s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    Aops = [cplx((m, k)) for _ in range(batch)]
    Bops = [cplx((k, n)) for _ in range(batch)]
    C0s = [cplx((m, n)) for _ in range(batch)]
    A = _slab([_stored(X, ta) for X in Aops], (k if ta != "N" else m) + 1)
    B = _slab([_stored(X, tb) for X in Bops], (n if tb != "N" else k) + 2)
    C = _slab(C0s, m + 3)
    alpha, beta = 0.5 + 1.5j, -1.25 - 0.5j
    oracle.zgemm_batched(ta, tb, m, n, k, alpha, A, B, beta, C)
    for i in range(batch):
        ref = alpha * (Aops[i] @ Bops[i]) + beta * C0s[i]
        assert np.linalg.norm(C[i, :, :m].T - ref) <= 1e-14 * np.linalg.norm(ref)


def test_batched_equals_single_threads_and_order():
    rng = np.random.default_rng(47)
    batch, m, n, k = 23, 10, 9, 14
    cplx = lambda s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    A = _slab([cplx((m, k)) for _ in range(batch)], m + 1)
    B = _slab([cplx((n, k)) for _ in range(batch)], n + 2)     # stored n x k, op 'C'
    C0 = _slab([cplx((m, n)) for _ in range(batch)], m)
    alpha, beta = 1.0 - 0.25j, 0.5j
    C1, C8 = C0.copy(), C0.copy()
    oracle.zgemm_batched("N", "C", m, n, k, alpha, A, B, beta, C1, nthreads=1)
    oracle.zgemm_batched("N", "C", m, n, k, alpha, A, B, beta, C8, nthreads=8)
    assert np.array_equal(C1.view(np.int64), C8.view(np.int64))
    # each instance is the single-instance product of its own operands
    for i in range(batch):
        Ci = C0[i].copy()
        assert oracle.zgemm("N", "C", m, n, k, alpha, A[i], m + 1, B[i], n + 2, beta, Ci, m) == 0
        assert np.array_equal(Ci.view(np.int64), C1[i].view(np.int64))
    # reversed pointer arrays give the same per-instance results
    rev = slice(None, None, -1)
    Ar, Br, Cr = (np.ascontiguousarray(X[rev]) for X in (A, B, C0))
    oracle.zgemm_batched("N", "C", m, n, k, alpha, Ar, Br, beta, Cr, nthreads=4)
    assert np.array_equal(Cr[rev].view(np.int64), C1.view(np.int64))


def test_batched_argument_rules():
    z = np.zeros((1, 2, 2), complex)
    with pytest.raises(ValueError):
        oracle.zgemm_batched("X", "N", 2, 2, 2, 1.0, z, z, 0.0, z.copy())
    with pytest.raises(ValueError):
        oracle.zgemm_batched("N", "N", 3, 2, 2, 1.0, z, z, 0.0, z.copy())   # lda 2 < m 3


ZB_MUTANTS = [
    ("other_instance_B",
     "int r = oracle_zgemm(transa, transb, m, n, k, alpha, A[i], lda, B[i], ldb,",
     "int r = oracle_zgemm(transa, transb, m, n, k, alpha, A[i], lda, B[0], ldb,"),
    ("swapped_lda_ldb",
     "int r = oracle_zgemm(transa, transb, m, n, k, alpha, A[i], lda, B[i], ldb,",
     "int r = oracle_zgemm(transa, transb, m, n, k, alpha, A[i], ldb, B[i], lda,"),
    ("dropped_last_instance",
     "    for (int i = 0; i < batch; ++i) {\n        int r = oracle_zgemm(",
     "    for (int i = 0; i < batch - 1; ++i) {\n        int r = oracle_zgemm("),
    ("beta_as_alpha",
     "                             beta, C[i], ldc);\n        if (r != 0) failed = 1;\n    }\n"
     "    return failed ? -100 : 0;\n}",
     "                             alpha, C[i], ldc);\n        if (r != 0) failed = 1;\n    }\n"
     "    return failed ? -100 : 0;\n}"),
]


def _build(text, d, name):
    c, so = os.path.join(d, name + ".c"), os.path.join(d, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-std=c99", c, "-o", so])
    return so


def _passes_in_child(so):
    code = ("import sys; import tests.test_oracle_zgemm_batched as t; "
            "sys.exit(0 if t._zb_pins_pass(t._load(sys.argv[1])) else 1)")
    r = subprocess.run([sys.executable, "-c", code, so], cwd=ROOT, capture_output=True,
                       timeout=120)
    return r.returncode == 0


def test_unmodified_batched_oracle_passes(tmp_path):
    with open(ORACLE_C) as f:
        assert _passes_in_child(_build(f.read(), str(tmp_path), "orig"))


@pytest.mark.parametrize("name,orig,mut", ZB_MUTANTS, ids=[z[0] for z in ZB_MUTANTS])
def test_batched_mutant_is_caught(tmp_path, name, orig, mut):
    with open(ORACLE_C) as f:
        src = f.read()
    assert src.count(orig) == 1, "mutation anchor not found: " + name
    assert not _passes_in_child(_build(src.replace(orig, mut), str(tmp_path), name))
