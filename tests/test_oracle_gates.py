"""Pins for the two-spin gate oracle (oracle/gates.py): the Kronecker-product
form on small states, norm preservation, U then U^H, a product state."""
import numpy as np
import pytest

from oracle import gates as G

rng = np.random.default_rng(41)


def _state(S):
    v = rng.standard_normal(1 << S) + 1j * rng.standard_normal(1 << S)
    return v / np.linalg.norm(v)


def _unitary():
    return G.haar_unitary(rng.standard_normal(16), rng.standard_normal(16))


@pytest.mark.parametrize("S,s", [(2, 0), (3, 0), (3, 1), (5, 2), (6, 4), (7, 0)])
def test_kronecker_form(S, s):
    # amplitude x = sum_j b_j 2^j: with numpy's kron (first factor varies
    # slowest), the operator is kron(I_high, U, I_low), U indexed by
    # q = b_s + 2 b_{s+1} -> in kron order the pair (b_{s+1}, b_s) is the
    # row-major index 2 b_{s+1} + b_s = q
    U = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    psi = _state(S)
    full = np.kron(np.kron(np.eye(1 << (S - s - 2)), U), np.eye(1 << s))
    ref = full @ psi
    got = G.apply_gate(psi, S, s, U)
    assert np.allclose(got, ref, rtol=0, atol=1e-14)


def test_members_partition_the_state():
    for S, s in [(4, 0), (4, 2), (9, 5)]:
        idx = G.members(S, s)
        assert sorted(idx.ravel().tolist()) == list(range(1 << S))


def test_unitary_preserves_norm_and_inverts():
    S = 10
    psi = _state(S)
    U = _unitary()
    assert np.allclose(U.conj().T @ U, np.eye(4), atol=1e-14)
    out = G.apply_gate(psi, S, 3, U)
    assert abs(np.linalg.norm(out) - 1.0) < 1e-14
    back = G.apply_gate(out, S, 3, U.conj().T)
    assert np.allclose(back, psi, atol=1e-14)


def test_product_state():
    S, s = 6, 2
    psi = np.zeros(1 << S, complex)
    psi[0] = 1.0
    U = _unitary()
    out = G.apply_gate(psi, S, s, U)
    # |0...0> maps to sum_q U[q, 0] |q at (s, s+1)>
    for q in range(4):
        x = ((q & 1) << s) | ((q >> 1) << (s + 1))
        assert out[x] == U[q, 0]
    assert np.count_nonzero(out) == 4
