"""GPU parity of the complex batched GEMM (bg_zgemm_batched) against the
complex oracle, through the C ABI: every op pair (N, T, C), tails in m, n and
k, padded leading dimensions with NaN canaries, complex alpha / beta, exact
Gaussian-integer results, the Hermitian Gram product at the paper's shapes,
and the scalar rules."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2203_09353_amd import bgemm, inputs

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def _zbatch(seed, stream, batch, rows, cols, ld, integer=False):
    re = inputs.uniform_batch(seed, 2 * stream, batch, rows, cols, ld)
    im = inputs.uniform_batch(seed, 2 * stream + 1, batch, rows, cols, ld)
    if integer:
        re, im = torch.round(re * 16), torch.round(im * 16)
    return torch.complex(re, im)


def _ordinary(S, rows, t):
    """(cols, ld) storage of a stored rows x cols matrix -> op() as an
    ordinary array."""
    X = S[:, :rows].T
    return X if t == "N" else (X.T if t == "T" else X.conj().T)


def run_case(h, ta, tb, m, n, k, alpha, beta, batch=3, pads=(0, 0, 0), seed=1, integer=False,
             c_nan=False):
    a_rows, a_cols = (m, k) if ta == "N" else (k, m)
    b_rows, b_cols = (k, n) if tb == "N" else (n, k)
    A = _zbatch(seed, 0, batch, a_rows, a_cols, max(1, a_rows + pads[0]), integer)
    B = _zbatch(seed, 1, batch, b_rows, b_cols, max(1, b_rows + pads[1]), integer)
    C = _zbatch(seed, 2, batch, m, n, max(1, m + pads[2]), integer)
    if c_nan:
        C[:, :, :m] = complex(float("nan"), float("nan"))
    Cd = C.cuda()
    h.zbatched(A.cuda(), B.cuda(), Cd, m, n, k, alpha, beta, ta, tb)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    An, Bn, Cn = A.numpy(), B.numpy(), C.numpy()
    ref = Cn.copy()
    oracle.zgemm_batched(ta, tb, m, n, k, alpha, An, Bn, beta, ref)
    # ld padding untouched, bit for bit
    assert np.array_equal(got[:, :, m:].view(np.int64), Cn[:, :, m:].view(np.int64))
    g = 2 * k * U / (1 - 2 * k * U)
    for i in range(batch):
        G, R = got[i, :, :m].T, ref[i, :, :m].T
        if integer:
            assert np.array_equal(G, R), (ta, tb, m, n, k, i)
            continue
        Aop, Bop = _ordinary(An[i], a_rows, ta), _ordinary(Bn[i], b_rows, tb)
        mag = (np.abs(Aop.real) + np.abs(Aop.imag)) @ (np.abs(Bop.real) + np.abs(Bop.imag))
        C0 = Cn[i, :, :m].T
        c0mag = 0.0 if beta == 0 else abs(beta) * (np.abs(C0.real) + np.abs(C0.imag))
        bound = (2 * g + 8 * U) * (abs(alpha) * 2 * mag + 2 * c0mag) + 1e-300
        assert np.all(np.abs(G - R) <= bound), (ta, tb, m, n, k, i)
        assert np.linalg.norm(G - R) <= 1e-13 * max(np.linalg.norm(R), 1e-300)


SHAPES = [(1, 1, 1), (7, 9, 13), (64, 64, 8), (65, 63, 17), (130, 129, 77), (33, 200, 5)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", list(itertools.product("NTC", "NTC")))
def test_complex_random(h, m, n, k, ta, tb):
    run_case(h, ta, tb, m, n, k, 1.0, 0.0, pads=(1, 2, 3))
    run_case(h, ta, tb, m, n, k, 0.75 - 1.25j, -0.5 + 2j, seed=2)


@pytest.mark.parametrize("ta,tb", list(itertools.product("NTC", "NTC")))
def test_complex_gaussian_integers_exact(h, ta, tb):
    run_case(h, ta, tb, 70, 45, 100, 2 - 1j, 1 + 3j, integer=True, pads=(2, 1, 0), seed=3)


@pytest.mark.parametrize("S", [13, 15])
def test_hermitian_gram_at_paper_shapes(h, S):
    # the entropy step forms Psi Psi^H for Psi of 2^ceil(S/2) x 2^floor(S/2)
    rows, cols = 2 ** ((S + 1) // 2), 2 ** (S // 2)
    Psi = _zbatch(4, 0, 2, rows, cols, rows)
    C = torch.zeros(2, rows, rows, dtype=torch.complex128)
    Cd = C.cuda()
    Pd = Psi.cuda()
    h.zbatched(Pd, Pd, Cd, rows, rows, cols, 1.0, 0.0, "N", "C")
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    ref = C.numpy().copy()
    oracle.zgemm_batched("N", "C", rows, rows, cols, 1.0, Psi.numpy(), Psi.numpy(), 0.0, ref)
    for i in range(2):
        G, R = got[i].T, ref[i].T
        assert np.linalg.norm(G - R) <= 1e-13 * np.linalg.norm(R)
        assert np.all(np.abs(np.diag(G).imag) <= 1e-13 * np.abs(np.diag(G).real))
        assert np.all(np.diag(G).real > 0)


def test_complex_scalar_rules(h):
    # beta == 0 never reads C (NaN canaries in C)
    run_case(h, "N", "N", 33, 31, 40, 1.0, 0.0, c_nan=True)
    A = _zbatch(5, 0, 2, 20, 30, 20)
    B = _zbatch(5, 1, 2, 30, 25, 30)
    C = _zbatch(5, 2, 2, 20, 25, 20)
    Ad, Bd = A.cuda(), B.cuda()
    # alpha == 0 with beta == 1: untouched bit for bit
    Cd = C.cuda()
    h.zbatched(Ad, Bd, Cd, 20, 25, 30, 0.0, 1.0)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu().view(torch.float64), C.view(torch.float64))
    # k == 0: C <- beta C; beta == 0 gives zeros without reading C
    Cd = C.cuda()
    h.zbatched(Ad, Bd, Cd, 20, 25, 0, 1.0, 0.5j)
    torch.cuda.synchronize()
    ref = C.numpy().copy()
    oracle.zgemm_batched("N", "N", 20, 25, 0, 1.0, A.numpy(), B.numpy(), 0.5j, ref)
    assert np.array_equal(Cd.cpu().numpy(), ref)
    Cn = C.clone()
    Cn[:, :, :] = complex(float("nan"), float("nan"))
    Cd = Cn.cuda()
    h.zbatched(Ad, Bd, Cd, 20, 25, 30, 0.0, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu(), torch.zeros_like(C))


def test_complex_argument_errors(h):
    A = _zbatch(6, 0, 1, 8, 8, 8).cuda()
    pA = bgemm.pointer_array(A)
    L = bgemm.lib()
    st = L.bg_zgemm_batched(h._h, b"N", b"N", 8, 8, 8, None, pA.data_ptr(), 8, pA.data_ptr(), 8,
                            None, pA.data_ptr(), 8, 1)
    assert st == 1 and h.last_invalid_arg() == 6
    with pytest.raises(bgemm.BgemmError) as e:
        h.zbatched(A, A, A.clone(), 8, 8, 8, 1.0, 0.0, "X", "N")
    assert e.value.arg == 1
    with pytest.raises(bgemm.BgemmError) as e:
        h.zbatched(A, A, A.clone(), 9, 8, 8, 1.0, 0.0, "N", "N")
    assert e.value.arg == 8


def test_hermitian_gram_s21_sampled_rows(h):
    # S = 21: Psi 2048 x 1024; 16 sampled rows of C against the oracle on
    # those rows of Psi (the same definition restricted to the rows)
    rows, cols = 2048, 1024
    Psi = _zbatch(7, 0, 1, rows, cols, rows)
    Pd = Psi.cuda()
    Cd = torch.zeros(1, rows, rows, dtype=torch.complex128, device="cuda")
    h.zbatched(Pd, Pd, Cd, rows, rows, cols, 1.0, 0.0, "N", "C")
    torch.cuda.synchronize()
    P = Psi.numpy()[0]
    sel = np.sort(np.random.default_rng(3).choice(rows, 16, replace=False))
    ref = np.zeros((1, rows, 16), dtype=np.complex128)
    oracle.zgemm_batched("N", "C", 16, rows, cols, 1.0, np.ascontiguousarray(P[:, sel])[None],
                         P[None], 0.0, ref)
    got = Cd.cpu().numpy()[0][:, sel]
    assert np.linalg.norm(got - ref[0]) <= 1e-13 * np.linalg.norm(ref[0])
