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

``i8emu<s>`` emulated binary64 with s int8 digit slices (s = 1..8), after
           Ozaki, Ogita, Oishi and Rump (Numer. Algorithms 59, 2012) with
           whole-row scaling and integer digit products, so that each
           diagonal is one exact integer sum over all of k:
    1. For row i of A, e_i is the exponent with max_p |A[i,p]| in
       [2^(e-1), 2^e) over all of k (frexp; 0 for an all-zero row); likewise
       f_j for column j of B.
    2. X[i,p] = rint(A[i,p] 2^(8s-2-e_i)) (ties to even), an integer with
       |X| <= 2^(8s-2); Y[p,j] likewise with f_j.
    3. Signed base-256 digits: X = sum_{t=1..s} d_t 256^(s-t) with
       d_t in [-128, 127] for t >= 2, taken from the least significant end
       (d_t = ((X + 128) mod 256) - 128, then X <- (X - d_t) / 256); what
       remains is d_1, in [-64, 64].  Every digit is an int8.
    4. For g = 2 .. s+1, S_g[i,j] = sum over t + u = g of
       sum_p dA_t[i,p] dB_u[p,j]: an exact integer (pairs with t + u > s + 1
       are dropped: s (s + 1) / 2 slice products).
    5. In binary64: T = S_{s+1}; for g = s down to 2: T = S_g + T 2^-8
       (rounded add; the scaled term is exact); V = T 2^(e_i + f_j - 12).
    6. C = alpha V + beta C (the binary64 rules).
  Truncation and dropped pairs bound the error by
  1.02 s k 2^(2-8s) 2^(e_i+f_j) per entry, the roundings of step 5 by about
  s u k 2^(e_i+f_j) (u = 2^-53).

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


def row_exponents(A):
    """e[i]: frexp exponent of max_p |A[i, p]| over the whole row (0 for an
    all-zero row)."""
    A = np.asarray(A, dtype=np.float64)
    mx = np.max(np.abs(A), axis=1) if A.shape[1] else np.zeros(A.shape[0])
    _, e = np.frexp(mx)
    return np.where(mx > 0, e, 0).astype(np.int64)


def int8_digits(X, s):
    """Signed base-256 digits d_1..d_s (int64 arrays, d_1 most significant)
    of the integers X, |X| <= 2^(8s-2), step 3 of the i8emu mode."""
    X = np.asarray(X, dtype=np.int64).copy()
    low = []
    for _ in range(s - 1):
        d = np.mod(X + 128, 256) - 128
        low.append(d)
        X = (X - d) // 256
    return [X] + low[::-1]


def int8_emulated_gemm(A, B, s, alpha=1.0, beta=0.0, C0=None):
    """The i8emu<s> mode, steps 1-6 above.  A (m, k), B (k, n) float64."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    e = row_exponents(A)
    f = row_exponents(B.T)
    X = np.rint(np.ldexp(A, (8 * s - 2) - e[:, None])).astype(np.int64)
    Y = np.rint(np.ldexp(B, (8 * s - 2) - f[None, :])).astype(np.int64)
    da = int8_digits(X, s)
    db = int8_digits(Y, s)
    S = {}
    for g in range(2, s + 2):
        acc = np.zeros((m, n), dtype=np.int64)
        for t in range(1, g):
            u = g - t
            if t <= s and u <= s:
                acc += da[t - 1] @ db[u - 1]                 # exact int64
        S[g] = acc
    T = S[s + 1].astype(np.float64)
    for g in range(s, 1, -1):
        T = S[g].astype(np.float64) + T * 2.0 ** -8
    V = np.ldexp(T, e[:, None] + f[None, :] - 12)
    if beta == 0.0:
        return alpha * V
    return alpha * V + beta * np.asarray(C0, dtype=np.float64)


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
