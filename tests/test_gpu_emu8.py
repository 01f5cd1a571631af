"""GPU parity of the int8-digit emulated binary64 mode (bg_gemm_batched_mode
with BG_MODE_EMU_I8) against the precision oracle, through the C ABI.

Every rounding of the mode is fixed (its diagonal sums are exact integers,
whatever the blocking of k), so the device must match
oracle.precision.int8_emulated_gemm bit for bit: every slice count, tile
tails in m, n and k, alpha / beta, exponent spreads of 2^+-20 and 2^+-300,
extreme digits, the largest supported k, and batches split into workspace
groups."""
import numpy as np
import pytest
import torch

from oracle import precision as P
from paper_2203_09353_amd import bgemm, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def _operands(seed, m, n, k, batch, pads, spread):
    lda, ldb, ldc = max(1, m + pads[0]), max(1, k + pads[1]), max(1, m + pads[2])
    A = inputs.uniform_batch(seed, 0, batch, m, k, lda)
    B = inputs.uniform_batch(seed, 1, batch, k, n, ldb)
    C = inputs.uniform_batch(seed, 2, batch, m, n, ldc)
    if spread:
        for X, st in ((A, 3), (B, 4)):
            E = torch.round(inputs.uniform_batch(seed, st, X.shape[0], X.shape[2], X.shape[1],
                                                 X.shape[2]) * spread)
            X.mul_(torch.exp2(torch.nan_to_num(E)))
    return A, B, C


def _mat(S, rows):
    return np.ascontiguousarray(S[:, :rows].T)


def _run(h, s, A, B, C, m, n, k, alpha=1.0, beta=0.0):
    Ad, Bd, Cd = A.cuda(), B.cuda(), C.cuda()
    h.batched_mode("i8emu", Ad, Bd, Cd, m, n, k, alpha, beta, slices=s)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    An, Bn, Cn = A.numpy(), B.numpy(), C.numpy()
    assert np.array_equal(got[:, :, m:].view(np.int64), Cn[:, :, m:].view(np.int64))
    return [(_mat(got[i], m), _mat(An[i], m), _mat(Bn[i], k), _mat(Cn[i], m))
            for i in range(C.shape[0])]


def _check(h, s, m, n, k, alpha=1.0, beta=0.0, batch=3, pads=(0, 0, 0), seed=5, spread=0):
    A, B, C = _operands(seed, m, n, k, batch, pads, spread)
    for G, Am, Bm, C0 in _run(h, s, A, B, C, m, n, k, alpha, beta):
        ref = P.int8_emulated_gemm(Am, Bm, s, alpha, beta, C0)
        assert np.array_equal(G.view(np.int64), ref.view(np.int64)), (s, m, n, k, alpha, beta)


@pytest.mark.parametrize("s", range(1, 9))
def test_i8_bit_exact_every_slice_count(h, s):
    _check(h, s, 70, 45, 100, pads=(3, 1, 2))


SHAPES = [(1, 1, 1), (64, 64, 64), (65, 63, 65), (130, 129, 77), (5, 200, 31), (128, 64, 256),
          (17, 3, 500)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("s", [3, 7])
def test_i8_bit_exact_shapes_alpha_beta(h, m, n, k, s):
    for alpha, beta, seed in ((1.0, 0.0, 6), (-0.75, 1.5, 7), (2.0, -1.0, 8)):
        _check(h, s, m, n, k, alpha, beta, batch=2, seed=seed)


@pytest.mark.parametrize("spread", [20, 300])
def test_i8_bit_exact_wide_exponents(h, spread):
    for s in (2, 5, 8):
        _check(h, s, 67, 66, 96, seed=11 + s, spread=spread)


def test_i8_extreme_digits_and_zero_lines(h):
    # entries next to their row's power of two give |X| = 2^(8s-2) (all-top
    # digits); zero rows of A and columns of B give exponent 0
    m, n, k = 48, 40, 130
    A, B, C = _operands(21, m, n, k, 2, (0, 0, 0), 0)
    g = torch.Generator().manual_seed(3)
    vals = torch.tensor([1 - 2.0 ** -53, -(1 - 2.0 ** -53), 0.5, -0.5, 0.5 + 2.0 ** -53,
                         0.75, -1 + 2.0 ** -40, 2.0 ** -60], dtype=torch.float64)
    for X in (A, B):
        idx = torch.randint(0, len(vals), X.shape, generator=g)
        X.copy_(vals[idx] * torch.exp2(torch.randint(-3, 4, X.shape, generator=g).double()))
    A[:, :, 5] = 0.0
    B[:, 7, :] = 0.0
    for s in (1, 4, 5, 7, 8):
        for G, Am, Bm, C0 in _run(h, s, A, B, C, m, n, k):
            ref = P.int8_emulated_gemm(Am, Bm, s)
            assert np.array_equal(G.view(np.int64), ref.view(np.int64)), s


def test_i8_largest_k(h):
    # k = 8192: the int32 diagonal sums are at their largest supported length
    A, B, C = _operands(23, 20, 18, 8192, 1, (0, 0, 0), 0)
    A[0, :, 3] = 1 - 2.0 ** -53          # a row of all-extreme digits
    B[0, 2, :] = -(1 - 2.0 ** -53)
    for G, Am, Bm, C0 in _run(h, 8, A, B, C, 20, 18, 8192):
        ref = P.int8_emulated_gemm(Am, Bm, 8)
        assert np.array_equal(G.view(np.int64), ref.view(np.int64))
    Ad, Bd, Cd = (torch.zeros(1, 8193, 4, dtype=torch.float64, device="cuda"),
                  torch.zeros(1, 4, 8193, dtype=torch.float64, device="cuda"),
                  torch.zeros(1, 4, 4, dtype=torch.float64, device="cuda"))
    with pytest.raises(bgemm.BgemmError) as e:
        h.batched_mode("i8emu", Ad, Bd, Cd, 4, 4, 8193, slices=7)
    assert e.value.status == 2


def test_i8_batches_in_workspace_groups():
    # a workspace for two instances' exponents: a batch of 5 runs in 3 groups
    m, n, k = 33, 31, 70
    hd = bgemm.Handle(workspace_bytes=2 * (m + n) * 4)
    try:
        A, B, C = _operands(25, m, n, k, 5, (1, 0, 2), 10)
        for G, Am, Bm, C0 in _run(hd, 6, A, B, C, m, n, k, 1.0, 0.5):
            ref = P.int8_emulated_gemm(Am, Bm, 6, 1.0, 0.5, C0)
            assert np.array_equal(G.view(np.int64), ref.view(np.int64))
        hd.set_workspace((m + n) * 4 - 4)
        with pytest.raises(bgemm.BgemmError) as e:
            _run(hd, 6, A, B, C, m, n, k)
        assert e.value.status == 4
    finally:
        hd.close()


def test_i8_accuracy_against_dot2(h):
    A, B, C = _operands(31, 64, 64, 256, 1, (0, 0, 0), 20)
    errs = []
    for s in (5, 6, 7, 8):
        G, Am, Bm, _ = _run(h, s, A, B, C, 64, 64, 256)[0]
        errs.append(P.relative_errors(G, P.dot2_gemm(Am, Bm))[0])
    fp64 = P.relative_errors(Am @ Bm, P.dot2_gemm(Am, Bm))[0]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 64, errs
    assert errs[2] < 1e-14 and errs[3] <= fp64, (errs, fp64)


def test_i8_scalar_rules_and_errors(h):
    A, B, C = _operands(61, 20, 30, 40, 2, (0, 0, 0), 0)
    Ad, Bd = A.cuda(), B.cuda()
    Cd = C.cuda()
    h.batched_mode("i8emu", Ad, Bd, Cd, 20, 30, 40, 0.0, 1.0, slices=4)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu().view(torch.int64), C.view(torch.int64))
    Cd = C.cuda()
    h.batched_mode("i8emu", Ad, Bd, Cd, 20, 30, 0, 1.0, -2.0, slices=4)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu()[:, :, :20], -2.0 * C[:, :, :20])
    Cn = C.clone()
    Cn[:, :, :20] = float("nan")
    Cd = Cn.cuda()
    h.batched_mode("i8emu", Ad, Bd, Cd, 20, 30, 40, 1.0, 0.0, slices=4)
    torch.cuda.synchronize()
    assert not torch.isnan(Cd.cpu()[:, :, :20]).any()
    for bad in (0, 9):
        with pytest.raises(bgemm.BgemmError) as e:
            h.batched_mode("i8emu", Ad, Bd, Cd, 20, 30, 40, slices=bad)
        assert e.value.status == 1 and e.value.arg == 102
    with pytest.raises(bgemm.BgemmError) as e:
        h.batched_mode("i8emu", Ad, Bd, Cd, 20, 30, 20, slices=3, transa="T")
    assert e.value.status == 2
