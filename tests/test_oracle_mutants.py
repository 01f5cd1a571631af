"""The oracle's pins have teeth: plant plausible mistakes in a copy of the
oracle's C source (on the CPU, in a temporary directory), build each mutant,
and check that the pin checks below reject every one of them while accepting
the unmodified source.  Each build is checked in a child process, since a
mutant with a wrong index may write out of bounds; a crash counts as caught."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ORACLE_C = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "oracle", "oracle.c")

# (name, original text, mutated text)
MUTANTS = [
    ("dropped_last_term", "for (int p = 0; p < k; ++p)", "for (int p = 0; p < k - 1; ++p)"),
    ("wrong_sign", "acc[r] = acc[r] + t;", "acc[r] = acc[r] - t;"),
    ("transposed_A_index", "A[(int64_t)r + (int64_t)p * slda]", "A[(int64_t)p + (int64_t)r * slda]"),
    ("transposed_B_index", "B[(int64_t)p + (int64_t)j * sldb]", "B[(int64_t)j + (int64_t)p * sldb]"),
    ("ignore_transb", "int ta = trans_code(transa), tb = trans_code(transb);\n    int64_t",
     "int ta = trans_code(transa), tb = 0;\n    int64_t"),
    ("beta_on_acc", "double y = beta * cj[r];", "double y = alpha * cj[r];"),
    ("reads_C_when_beta0", "cj[r] = use_product ? alpha * acc[r] : 0.0;",
     "cj[r] = use_product ? alpha * acc[r] + 0.0 * cj[r] : 0.0;"),
    ("ldc_as_m", "double *cj = C + (int64_t)j * sldc;", "double *cj = C + (int64_t)j * m;"),
    ("beta1_scales", "if (beta != 1.0) cj[r] = beta * cj[r];", "cj[r] = beta * cj[r] + 0.0;"),
    ("skip_k0_check", "int use_product = !(alpha == 0.0 || k == 0);", "int use_product = 1;"),
    ("lda_check_off", "if (lda < imax1(ta ? k : m)) return -8;", "if (lda < 1) return -8;"),
]


def _build(src_text, d, name):
    c = os.path.join(d, name + ".c")
    so = os.path.join(d, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-std=c99", c, "-o", so])
    return so


def _load(so):
    L = ctypes.CDLL(so)
    L.oracle_dgemm.restype = ctypes.c_int
    L.oracle_dgemm.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p,
                               ctypes.c_int]
    return L


def _call(L, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    return L.oracle_dgemm(ta.encode(), tb.encode(), m, n, k, alpha, A.ctypes.data, lda,
                          B.ctypes.data, ldb, beta, C.ctypes.data, ldc)


def _pins_pass(L):
    """A compact selection of the pins: integer exactness for all transposes
    with padded leading dimensions, NaN canaries, beta == 1 bit-identity,
    k == 0, and the lda rule."""
    rng = np.random.default_rng(5)
    m, n, k = 9, 7, 11
    Ai = rng.integers(-32, 33, (m, k)); Bi = rng.integers(-32, 33, (k, n))
    C0 = rng.integers(-32, 33, (m, n)).astype(float)
    for ta in "NT":
        for tb in "NT":
            A = Ai.T if ta == "T" else Ai
            B = Bi.T if tb == "T" else Bi
            lda, ldb, ldc = A.shape[0] + 2, B.shape[0] + 3, m + 1
            As = np.full((A.shape[1], lda), np.nan); As[:, :A.shape[0]] = A.T
            Bs = np.full((B.shape[1], ldb), np.nan); Bs[:, :B.shape[0]] = B.T
            for alpha, beta in [(1.0, 0.0), (2.0, -0.5)]:
                Cs = np.full((n, ldc), np.nan)
                Cs[:, :m] = C0.T if beta != 0 else np.nan
                if _call(L, ta, tb, m, n, k, alpha, As, lda, Bs, ldb, beta, Cs, ldc) != 0:
                    return False
                exp = alpha * (Ai @ Bi).astype(float) + (beta * C0 if beta != 0 else 0.0)
                if not np.array_equal(Cs[:, :m].T, exp):
                    return False
                if not np.isnan(Cs[:, m:]).all():
                    return False
    # beta == 1 with k == 0 leaves C bit-identical; beta == 0.5 with k == 0 scales
    Cs = rng.uniform(-1, 1, (n, m)); Cs[0, 0] = -0.0; before = Cs.copy()
    z = np.zeros(1)
    if _call(L, "N", "N", m, n, 0, 1.0, z, m, z, 1, 1.0, Cs, m) != 0:
        return False
    if not np.array_equal(Cs.view(np.int64), before.view(np.int64)):
        return False
    if _call(L, "N", "N", m, n, 0, 1.0, z, m, z, 1, 0.5, Cs, m) != 0:
        return False
    if not np.array_equal(Cs, 0.5 * before):
        return False
    # the lda rule
    if _call(L, "N", "N", 4, 1, 2, 1.0, z, 3, z, 2, 0.0, z, 4) != -8:
        return False
    return True


@pytest.fixture(scope="module")
def source():
    with open(ORACLE_C) as f:
        return f.read()


def _passes_in_child(so):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; import tests.test_oracle_mutants as t; "
            "sys.exit(0 if t._pins_pass(t._load(sys.argv[1])) else 1)")
    r = subprocess.run([sys.executable, "-c", code, so], cwd=root, capture_output=True,
                       timeout=120)
    return r.returncode == 0


def test_unmodified_oracle_passes(source, tmp_path):
    assert _passes_in_child(_build(source, str(tmp_path), "orig"))


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, tmp_path, name, orig, mut):
    assert source.count(orig) == 1, "mutation anchor not found: " + name
    so = _build(source.replace(orig, mut), str(tmp_path), name)
    assert not _passes_in_child(so), "pins did not catch mutant " + name
