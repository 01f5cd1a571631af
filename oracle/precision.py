"""CPU oracle for the reduced- and emulated-precision GEMM modes -- TEST
INFRASTRUCTURE ONLY (tests, smoke and the benchmark's CPU leg).

These modes compute the same product as the paper's Eq. 1 (Section II),
C <- alpha A B + beta C, through cheaper arithmetic; each mode is defined here
step by step, plainly, in float64 / int64 numpy (matrices as ordinary
(rows, cols) arrays, no transposes: op(X) = X).

Modes
-----
``fp32``   A and B rounded to binary32 (round to nearest even); their product
           accumulated in binary32 by the device; alpha/beta in binary64.
           The reference here is the product of the rounded inputs in
           binary64; a device result is correct within binary32 accumulation
           error (Higham's gamma_k with u = 2^-24).
``bf16``   A and B rounded to binary32 and then to bfloat16 (both round to
           nearest even: the device converts through binary32), products
           accumulated in binary32.  Same kind of reference and tolerance.
``emu<s>`` emulated binary64 with s bfloat16 digit slices (s = 1..8).  Defined
           as follows (all steps exact unless marked "rounded"):
    1. k is cut into chunks of 32 (the last one may be shorter).  For row i
       of A and chunk c, e_ic is the exponent with max_p |A[i,p]| in
       [2^(e-1), 2^e) over the chunk (frexp; 0 for an all-zero row part);
       likewise f_jc for column j of B.  Scaled values x = A[i,p] 2^-e_ic and
       y = B[p,j] 2^-f_jc lie in (-1, 1).
    2. Digits of x in (-1, 1): d_1 = rint(x 2^7), r_1 = x 2^7 - d_1, and for
       t >= 2: d_t = rint(r_{t-1} 2^8), r_t = r_{t-1} 2^8 - d_t (rint: to
       nearest, ties to even).  Every digit is an integer in [-128, 128]
       (exact in bfloat16), every remainder lies in [-1/2, 1/2], and
       x = sum_{t<=s} d_t 2^(-7-8(t-1)) + r_s 2^(-7-8(s-1)).
    3. For each diagonal g = 2 .. s+1, S_gc[i,j] = sum over slice pairs
       t + u = g (t, u >= 1) of sum_{p in chunk c} dA_t[i,p] dB_u[p,j]: an
       integer of magnitude <= g * 32 * 2^14 < 2^24, exact in binary32
       accumulation whatever the order.  Pairs with t + u > s + 1 are dropped
       (s (s + 1) / 2 slice products per chunk).
    4. Per chunk, in binary64: T = 0; for g = s+1 down to 2:
       T = T + S_gc 2^(-14-8(g-2))  (rounded add; the scaled term is exact),
       then V_c = T 2^(e_ic + f_jc).
    5. acc = 0; for chunks c ascending: acc = acc + V_c (rounded).
    6. C = alpha acc + beta C (as the binary64 path: alpha acc and beta C each
       rounded, then a rounded add; beta = 0 never reads C).
  Since every rounding is fixed in kind and order, a device implementing
  these steps must match this oracle bit for bit.

Error reference
---------------
``dot2_gemm`` is the compensated product of Ogita, Rump and Oishi ("Accurate
sum and dot product", SIAM J. Sci. Comput. 26(6), 2005, algorithm Dot2):
each entry is computed as if in twice binary64 precision and then rounded, so
the error of the binary64 oracle itself becomes visible beside a mode's error.
Error-free transformations: TwoSum (Knuth) and TwoProduct (Dekker, with
Veltkamp's split by 2^27 + 1; valid while |entries| stay below about 2^995).

Parity status: every function is pinned in tests/test_oracle_precision.py.
"""
from __future__ import annotations

import numpy as np

CHUNK = 32


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """binary64 -> binary32 -> bfloat16, each round to nearest even."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    # round to nearest even on the top 16 bits (finite inputs)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def reference_product(A, B, mode):
    """binary64 product of the rounded inputs of mode 'fp32' or 'bf16'."""
    rnd = round_fp32 if mode == "fp32" else round_bf16
    return rnd(A) @ rnd(B)


def chunk_exponents_rows(A, c0, c1):
    """e[i]: frexp exponent of max |A[i, c0:c1]| (0 for all-zero)."""
    mx = np.max(np.abs(A[:, c0:c1]), axis=1) if c1 > c0 else np.zeros(A.shape[0])
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, 0).astype(np.int64)


def digits(x, s):
    """Digits d_1..d_s (int64 arrays) and the last remainder of x in (-1, 1)."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    r = x * 128.0
    for t in range(s):
        d = np.rint(r)
        out.append(d.astype(np.int64))
        r = (r - d) * 256.0
    return out, r / 256.0


def emulated_gemm(A, B, s, alpha=1.0, beta=0.0, C0=None):
    """The emu<s> mode, steps 1-6 above.  A (m, k), B (k, n) float64."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    acc = np.zeros((m, n))
    for c0 in range(0, k, CHUNK):
        c1 = min(k, c0 + CHUNK)
        e = chunk_exponents_rows(A, c0, c1)                  # (m,)
        f = chunk_exponents_rows(B.T, c0, c1)                # (n,)
        xa = np.ldexp(A[:, c0:c1], -e[:, None])
        yb = np.ldexp(B[c0:c1, :], -f[None, :])
        da, _ = digits(xa, s)
        db, _ = digits(yb, s)
        T = np.zeros((m, n))
        for g in range(s + 1, 1, -1):
            S = np.zeros((m, n), dtype=np.int64)
            for t in range(1, g):
                u = g - t
                if t > s or u > s:
                    continue
                S += da[t - 1] @ db[u - 1]                   # exact int64
            T = T + np.ldexp(S.astype(np.float64), -14 - 8 * (g - 2))
        V = np.ldexp(T, e[:, None] + f[None, :])
        acc = acc + V
    if beta == 0.0:
        return alpha * acc
    return alpha * acc + beta * np.asarray(C0, dtype=np.float64)


def _two_sum(a, b):
    s = a + b
    z = s - a
    return s, (a - (s - z)) + (b - z)


def _split(a):
    c = 134217729.0 * a          # 2^27 + 1
    hi = c - (c - a)
    return hi, a - hi


def _two_product(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, al * bl - (((p - ah * bh) - al * bh) - ah * bl)


def dot2_gemm(A, B):
    """A B with every entry from Dot2 over p ascending (binary64 result)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    if k == 0:
        return np.zeros((m, n))
    p, s = _two_product(A[:, :1], B[:1, :])
    for q in range(1, k):
        h, r = _two_product(A[:, q:q + 1], B[q:q + 1, :])
        p, e = _two_sum(p, h)
        s = s + (e + r)
    return p + s


def relative_errors(C, ref):
    """Per-instance relative Frobenius error and max elementwise relative error
    (to max |ref| of the instance)."""
    C = np.asarray(C); ref = np.asarray(ref)
    fro = np.linalg.norm(C - ref) / max(np.linalg.norm(ref), 1e-300)
    mx = np.max(np.abs(C - ref)) / max(np.max(np.abs(ref)), 1e-300)
    return fro, mx
