"""Parity helpers: run the CPU oracle on host copies of the same seeded
inputs and compare the GPU result against it, instance by instance.

Tolerances (FP64 paths):
  * integer-valued inputs whose partial sums are exact in binary64: the
    results must be equal (bit-exact up to the sign of zero);
  * otherwise, per instance, ||C_gpu - C_ref||_F <= 1e-13 ||C_ref||_F, and
    elementwise |C_gpu - C_ref| <= (2 gamma_k + 4u) (|alpha| |op A||op B| +
    |beta| |C0|) + tiny, since both results obey Higham's bound
    |fl(AB) - AB| <= gamma_k |A||B| (Accuracy and Stability of Numerical
    Algorithms, Section 3.5) plus the roundings of the alpha/beta update.
"""
import numpy as np

import oracle
from tests.colmajor import U, gamma

REL_FRO = 1e-13
TINY = 1e-300


def op_view(S, rows, cols, t):
    """(cols_stored, ld) storage of a stored rows x cols matrix -> op() as an
    ordinary (rows_op, cols_op) array."""
    X = S[:cols, :rows].T
    return X.T if t in "TtCc" else X


def check_instance(got, ref, Aop, Bop, C0, alpha, beta, exact=False, where=""):
    """got, ref, C0: (m, n) arrays; Aop (m, k), Bop (k, n) ordinary arrays."""
    if exact:
        bad = ~((got == ref) | (np.isnan(got) & np.isnan(ref)))
        assert not bad.any(), "%s: %d elements differ (exact), first at %s: %r vs %r" % (
            where, int(bad.sum()), np.argwhere(bad)[0], got[bad][0], ref[bad][0])
        return
    assert np.isfinite(got).all(), where + ": non-finite result"
    d = np.linalg.norm(got - ref)
    r = np.linalg.norm(ref)
    assert d <= REL_FRO * r or (r == 0 and d == 0), "%s: rel Frobenius %.3e" % (
        where, d / r if r else np.inf)
    k = Aop.shape[1]
    scale = abs(alpha) * (np.abs(Aop) @ np.abs(Bop)) if k else 0.0
    if beta != 0:
        scale = scale + abs(beta) * np.abs(C0)
    bound = (2 * gamma(max(k, 1)) + 4 * U) * scale + TINY
    err = np.abs(got - ref)
    bad = err > bound
    assert not bad.any(), "%s: %d elements above the componentwise bound" % (where, int(bad.sum()))


def oracle_uniform(ta, tb, m, n, k, alpha, A, B, beta, C0):
    """A, B, C0: host (batch, cols, ld) arrays; returns the oracle's C."""
    C = np.ascontiguousarray(C0.copy())
    oracle.gemm_batched(ta, tb, m, n, k, alpha, np.ascontiguousarray(A), np.ascontiguousarray(B),
                        beta, C)
    return C
