"""Two-spin gates on S-spin states, plain numpy -- TEST INFRASTRUCTURE ONLY
(tests, smoke and the benchmark's CPU leg).

The paper's Monte Carlo step applies a local unitary to a randomly chosen
pair of neighbouring spins of a 2^S-amplitude state (Section III, Alg. 1)
and gives no gate model; here a gate is any 4 x 4 complex matrix U.
Amplitude x (0 <= x < 2^S) has spin j in bit j of x.  A gate on spins
(s, s + 1) acts on every quadruple of amplitudes that differ only in those
two bits: with local index q = b_s + 2 b_{s+1},
    psi'[x0 + q-th member] = sum over q' of U[q, q'] psi[x0 + q'-th member]
(each output a plain complex dot product of length 4, q' ascending; every
complex product (u, v) -> (u_re v_re - u_im v_im, u_re v_im + u_im v_re) and
every add rounded).  U is stored column-major: U[q, q'] at 4 q' + q.

Parity status: pinned in tests/test_oracle_gates.py (the Kronecker-product
form kron(I, U, I) on small S, norm preservation by unitaries, U then U^H,
a product state).
"""
from __future__ import annotations

import numpy as np


def members(S: int, s: int) -> np.ndarray:
    """(2^(S-2), 4) amplitude indices of every quadruple, local order q."""
    g = np.arange(1 << (S - 2), dtype=np.int64)
    low = g & ((1 << s) - 1)
    x0 = low | ((g >> s) << (s + 2))
    q = np.arange(4, dtype=np.int64)
    return x0[:, None] + ((q & 1) << s)[None, :] + ((q >> 1) << (s + 1))[None, :]


def apply_gate(psi: np.ndarray, S: int, s: int, U: np.ndarray) -> np.ndarray:
    """psi: complex128 vector of 2^S amplitudes; U: (4, 4) complex128 (ordinary
    indexing U[q, q']).  Returns the new state (a copy)."""
    idx = members(S, s)
    v = psi[idx]                                   # (groups, 4)
    out_re = np.zeros(v.shape)
    out_im = np.zeros(v.shape)
    for q in range(4):
        acc_re = np.zeros(v.shape[0])
        acc_im = np.zeros(v.shape[0])
        for qp in range(4):
            u = U[q, qp]
            pr = u.real * v[:, qp].real - u.imag * v[:, qp].imag
            pi = u.real * v[:, qp].imag + u.imag * v[:, qp].real
            acc_re = acc_re + pr
            acc_im = acc_im + pi
        out_re[:, q] = acc_re
        out_im[:, q] = acc_im
    res = psi.copy()
    res[idx] = out_re + 1j * out_im
    return res


def haar_unitary(rng_values_re: np.ndarray, rng_values_im: np.ndarray) -> np.ndarray:
    """4 x 4 Haar unitary from 16 + 16 standard normal values (QR with the
    sign fix of Mezzadri)."""
    Z = (np.asarray(rng_values_re).reshape(4, 4) + 1j * np.asarray(rng_values_im).reshape(4, 4))
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]
