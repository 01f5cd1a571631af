"""Small helpers for tests: convert between ordinary (rows, cols) numpy
matrices and the column-major storage used by the oracle and the library,
an array of shape (cols, ld) whose first ``rows`` entries per column hold the
matrix and whose padding rows hold NaN."""
import numpy as np


def store(X, ld=None, pad=np.nan):
    """(rows, cols) matrix -> (cols, ld) column-major storage."""
    X = np.asarray(X, dtype=np.float64)
    rows, cols = X.shape
    ld = max(rows, 1) if ld is None else ld
    out = np.full((cols, ld), pad, dtype=np.float64)
    out[:, :rows] = X.T
    return out


def load(S, rows):
    """(cols, ld) column-major storage -> (rows, cols) matrix."""
    return np.ascontiguousarray(S[:, :rows].T)


def op(X, t):
    return X.T if t in "TtCc" else X


def rel_frobenius(X, ref):
    d = np.linalg.norm(np.asarray(X) - np.asarray(ref))
    r = np.linalg.norm(np.asarray(ref))
    if r == 0.0:
        return 0.0 if d == 0.0 else np.inf
    return d / r


U = 2.0 ** -53


def gamma(n):
    """Higham's gamma_n = n u / (1 - n u), u the unit roundoff of binary64."""
    return n * U / (1.0 - n * U)
