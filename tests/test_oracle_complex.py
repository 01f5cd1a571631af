"""Pins for the complex oracle (oracle_zgemm in oracle/oracle.c): numpy's
complex matmul on random data for every op pair, exact results on
Gaussian-integer data against Python integer arithmetic, the Hermitian
structure of a Gram product, the scalar rules, and mutants of the complex code
that these pins must reject."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPS = [(a, b) for a in "NTC" for b in "NTC"]


def _op(X, t):
    return X if t == "N" else (X.T if t == "T" else X.conj().T)


def _store(X, ld, fill=np.nan):
    """Ordinary (rows, cols) complex matrix -> (cols, ld) column-major storage."""
    S = np.full((X.shape[1], ld), complex(fill, fill))
    S[:, :X.shape[0]] = X.T
    return S


def _run(ta, tb, Aop, Bop, alpha, beta, C0, pads=(1, 2, 3), lib=None):
    """Calls the oracle on op(A) = Aop, op(B) = Bop (stored per ta / tb)."""
    m, k = Aop.shape
    n = Bop.shape[1]
    A = _op(Aop, ta) if ta != "C" else Aop.conj().T        # stored matrix
    B = _op(Bop, tb) if tb != "C" else Bop.conj().T
    As, Bs = _store(A, A.shape[0] + pads[0]), _store(B, B.shape[0] + pads[1])
    Cs = _store(C0, m + pads[2])
    if lib is None:
        r = oracle.zgemm(ta, tb, m, n, k, alpha, As, As.shape[1], Bs, Bs.shape[1], beta, Cs,
                         Cs.shape[1])
    else:
        pair = lambda z: (ctypes.c_double * 2)(complex(z).real, complex(z).imag)
        r = lib.oracle_zgemm(ta.encode(), tb.encode(), m, n, k, pair(alpha), As.ctypes.data,
                             As.shape[1], Bs.ctypes.data, Bs.shape[1], pair(beta), Cs.ctypes.data,
                             Cs.shape[1])
    return r, Cs


rng = np.random.default_rng(23)


def _cplx(shape, ints=False):
    if ints:
        return (rng.integers(-16, 17, shape) + 1j * rng.integers(-16, 17, shape)).astype(complex)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("ta,tb", OPS)
def test_against_numpy(ta, tb):
    m, n, k = 13, 9, 21
    Aop, Bop, C0 = _cplx((m, k)), _cplx((k, n)), _cplx((m, n))
    alpha, beta = 0.75 - 1.25j, -0.5 + 2j
    r, Cs = _run(ta, tb, Aop, Bop, alpha, beta, C0)
    assert r == 0
    ref = alpha * (Aop @ Bop) + beta * C0
    got = Cs[:, :m].T
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    assert np.isnan(Cs[:, m:].real).all()            # ld padding untouched


def _exact_int(Aop, Bop, alpha, beta, C0):
    """Python integer arithmetic on Gaussian integers."""
    m, k = Aop.shape
    n = Bop.shape[1]
    out = np.zeros((m, n), complex)
    for i in range(m):
        for j in range(n):
            sr = si = 0
            for p in range(k):
                ar, ai = int(Aop[i, p].real), int(Aop[i, p].imag)
                br, bi = int(Bop[p, j].real), int(Bop[p, j].imag)
                sr += ar * br - ai * bi
                si += ar * bi + ai * br
            xr = int(alpha.real) * sr - int(alpha.imag) * si
            xi = int(alpha.real) * si + int(alpha.imag) * sr
            cr, ci = int(C0[i, j].real), int(C0[i, j].imag)
            yr = int(beta.real) * cr - int(beta.imag) * ci
            yi = int(beta.real) * ci + int(beta.imag) * cr
            out[i, j] = complex(xr + yr, xi + yi)
    return out


def _zpins_pass(lib=None):
    m, n, k = 6, 5, 9
    for ta, tb in OPS:
        Aop, Bop, C0 = _cplx((m, k), True), _cplx((k, n), True), _cplx((m, n), True)
        for alpha, beta in ((1 + 0j, 0j), (2 - 1j, 1 + 3j)):
            Cin = C0 if beta != 0 else np.full((m, n), complex(np.nan, np.nan))
            r, Cs = _run(ta, tb, Aop, Bop, alpha, beta, Cin, lib=lib)
            if r != 0:
                return False
            exp = _exact_int(Aop, Bop, alpha, beta, C0 if beta != 0 else np.zeros((m, n)))
            if not np.array_equal(Cs[:, :m].T, exp):
                return False
            if not np.isnan(Cs[:, m:].real).all():
                return False
    # alpha == 0 with beta == 1: C untouched bit for bit; k == 0 scales
    C0 = _cplx((m, n))
    r, Cs = _run("N", "N", np.zeros((m, 0)), np.zeros((0, n)), 1.0, 1.0, C0, lib=lib)
    if r != 0 or not np.array_equal(np.ascontiguousarray(Cs[:, :m].T).view(np.int64),
                                    C0.view(np.int64)):
        return False
    r, Cs = _run("N", "N", _cplx((m, k)), _cplx((k, n)), 0.0, 0.5j, C0, lib=lib)
    if r != 0 or not np.array_equal(Cs[:, :m].T, 0.5j * C0):
        return False
    return True


def test_gaussian_integers_exact_and_scalar_rules():
    assert _zpins_pass()


@pytest.mark.parametrize("m,k", [(7, 3), (16, 31)])
def test_hermitian_gram_product(m, k):
    # C = Psi Psi^H: the diagonal's imaginary part is exactly zero (each term
    # pair a_im a_re - a_re a_im cancels exactly on a zero running sum), its
    # real part is a sum of squares; mirrored entries agree to rounding
    Psi = _cplx((m, k))
    r, Cs = _run("N", "C", Psi, Psi.conj().T, 1.0, 0.0, np.zeros((m, m)), pads=(0, 0, 0))
    C = Cs.T
    assert r == 0
    assert np.all(np.diag(C).imag == 0) and np.all(np.diag(C).real >= 0)
    mag = np.abs(Psi.real) @ np.abs(Psi.real).T + np.abs(Psi.imag) @ np.abs(Psi.imag).T + \
        np.abs(Psi.imag) @ np.abs(Psi.real).T + np.abs(Psi.real) @ np.abs(Psi.imag).T
    g = 2 * k * 2.0 ** -53 / (1 - 2 * k * 2.0 ** -53)
    assert np.all(np.abs(C - C.conj().T) <= 2 * g * mag)
    ref = Psi @ Psi.conj().T
    assert np.linalg.norm(C - ref) <= 1e-14 * np.linalg.norm(ref)


def test_transpose_and_conjugate_differ():
    Aop, Bop = _cplx((4, 5)), _cplx((5, 3))
    _, c1 = _run("T", "N", Aop, Bop, 1.0, 0.0, np.zeros((4, 3)))
    _, c2 = _run("C", "N", Aop, Bop, 1.0, 0.0, np.zeros((4, 3)))
    # both compute op(A) op(B) for the op(A) given: equal results, different storage read
    assert np.allclose(c1[:, :4], c2[:, :4])
    A = _cplx((5, 4))
    As = _store(A, 5, 0)
    C1 = np.zeros((3, 4), complex); C2 = np.zeros((3, 4), complex)
    Bs = _store(Bop, 5, 0)
    oracle.zgemm("T", "N", 4, 3, 5, 1.0, As, 5, Bs, 5, 0.0, C1, 4)
    oracle.zgemm("C", "N", 4, 3, 5, 1.0, As, 5, Bs, 5, 0.0, C2, 4)
    assert np.allclose(C1.T, A.T @ Bop) and np.allclose(C2.T, A.conj().T @ Bop)
    assert not np.allclose(C1, C2)


ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
ZMUTANTS = [
    ("dropped_conj_a", "double are = ap[0], aim = ta == 2 ? -ap[1] : ap[1];",
     "double are = ap[0], aim = ap[1];"),
    ("dropped_conj_b", "double bre = bp[0], bim = tb == 2 ? -bp[1] : bp[1];",
     "double bre = bp[0], bim = bp[1];"),
    ("im_im_sign", "t = (-aim) * bim;", "t = aim * bim;"),
    ("swapped_cross_term", "t = aim * bre;", "t = aim * bim;"),
    ("alpha_im_sign", "double xr = ar_ * acc[2 * r] - ai_ * acc[2 * r + 1];",
     "double xr = ar_ * acc[2 * r] + ai_ * acc[2 * r + 1];"),
    ("reads_C_when_beta0", "if (beta_zero) { c[0] = xr; c[1] = xi; continue; }",
     "if (0) { c[0] = xr; c[1] = xi; continue; }"),
    ("ldc_real_stride", "double *cj = C + 2 * (int64_t)j * sldc;", "double *cj = C + (int64_t)j * sldc;"),
    ("t_conjugates", "if (t == 'T' || t == 't') return 1;", "if (t == 'T' || t == 't') return 2;"),
]


def _load(so):
    L = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_zgemm.restype = ctypes.c_int
    L.oracle_zgemm.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, dp, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                               ctypes.c_int, dp, ctypes.c_void_p, ctypes.c_int]
    return L


def _passes_in_child(so):
    code = ("import sys; import tests.test_oracle_complex as t; "
            "sys.exit(0 if t._zpins_pass(t._load(sys.argv[1])) else 1)")
    r = subprocess.run([sys.executable, "-c", code, so], cwd=ROOT, capture_output=True,
                       timeout=120)
    return r.returncode == 0


def _build(text, d, name):
    c, so = os.path.join(d, name + ".c"), os.path.join(d, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-std=c99", c, "-o", so])
    return so


def test_unmodified_complex_oracle_passes(tmp_path):
    with open(ORACLE_C) as f:
        assert _passes_in_child(_build(f.read(), str(tmp_path), "orig"))


@pytest.mark.parametrize("name,orig,mut", ZMUTANTS, ids=[z[0] for z in ZMUTANTS])
def test_complex_mutant_is_caught(tmp_path, name, orig, mut):
    with open(ORACLE_C) as f:
        src = f.read()
    assert src.count(orig) == 1, "mutation anchor not found: " + name
    assert not _passes_in_child(_build(src.replace(orig, mut), str(tmp_path), name))
