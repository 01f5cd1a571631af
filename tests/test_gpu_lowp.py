"""GPU parity of the reduced- and emulated-precision modes of the uniform
batch (bg_gemm_batched_mode) against the precision oracle
(oracle/precision.py), through the C ABI.

The emulated mode fixes every rounding, so it must match the oracle bit for
bit, whatever the slice count, tile tails, exponent spread or alpha / beta.
The fp32 and bf16 modes are checked against the binary64 product of the
rounded inputs within binary32 accumulation error, and against the binary64
result with a lower bound on the error (the reduced arithmetic really ran)."""
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
    """Column-major storage (batch, cols, ld) with NaN padding rows; entries
    uniform in [-1, 1) times 2^E with E uniform on the integers of
    [-spread, spread] (a second seeded stream)."""
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


def run_mode(h, mode, slices, m, n, k, alpha=1.0, beta=0.0, batch=3, pads=(0, 0, 0), seed=5,
             spread=0):
    A, B, C = _operands(seed, m, n, k, batch, pads, spread)
    Ad, Bd, Cd = A.cuda(), B.cuda(), C.cuda()
    h.batched_mode(mode, Ad, Bd, Cd, m, n, k, alpha, beta, slices=slices)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    An, Bn, Cn = A.numpy(), B.numpy(), C.numpy()
    # padding rows untouched, bit for bit
    assert np.array_equal(got[:, :, m:].view(np.int64), Cn[:, :, m:].view(np.int64))
    out = []
    for i in range(batch):
        Am, Bm, C0 = _mat(An[i], m), _mat(Bn[i], k), _mat(Cn[i], m)
        out.append((_mat(got[i], m), Am, Bm, C0))
    return out


@pytest.mark.parametrize("s", range(1, 9))
def test_emulated_bit_exact_every_slice_count(h, s):
    for G, Am, Bm, C0 in run_mode(h, "emu", s, 70, 45, 100, pads=(3, 1, 2)):
        ref = P.emulated_gemm(Am, Bm, s)
        assert np.array_equal(G.view(np.int64), ref.view(np.int64)), s


EMU_SHAPES = [(1, 1, 1), (64, 64, 32), (65, 63, 33), (130, 129, 77), (5, 200, 31),
              (128, 64, 256), (17, 3, 500)]


@pytest.mark.parametrize("m,n,k", EMU_SHAPES)
@pytest.mark.parametrize("s", [3, 7])
def test_emulated_bit_exact_shapes_alpha_beta(h, m, n, k, s):
    for alpha, beta, seed in ((1.0, 0.0, 6), (-0.75, 1.5, 7), (2.0, -1.0, 8)):
        for G, Am, Bm, C0 in run_mode(h, "emu", s, m, n, k, alpha, beta, seed=seed, batch=2):
            ref = P.emulated_gemm(Am, Bm, s, alpha, beta, C0)
            assert np.array_equal(G.view(np.int64), ref.view(np.int64)), (m, n, k, s, alpha, beta)


@pytest.mark.parametrize("spread", [20, 300])
def test_emulated_bit_exact_wide_exponents(h, spread):
    # per-chunk scaling with entries far below their chunk's largest one
    for s in (2, 5, 8):
        for G, Am, Bm, C0 in run_mode(h, "emu", s, 67, 66, 96, seed=11 + s, spread=spread):
            ref = P.emulated_gemm(Am, Bm, s)
            assert np.array_equal(G.view(np.int64), ref.view(np.int64)), (spread, s)


@pytest.mark.parametrize("s", [1, 3, 6, 8])
def test_emulated_on_binary32_cores_bit_exact(h, s):
    """BG_MODE_EMU_F32: the same digits summed on the binary32 matrix cores
    give the oracle's bits (and so the bfloat16-core mode's), with tails in m,
    n and k, padding, alpha / beta and a wide exponent spread."""
    for m, n, k, alpha, beta, spread in ((70, 45, 100, 1.0, 0.0, 0), (65, 63, 33, -0.75, 1.5, 0),
                                         (17, 3, 500, 2.0, -1.0, 20)):
        res = run_mode(h, "f32emu", s, m, n, k, alpha, beta, pads=(3, 1, 2), seed=40 + s,
                       spread=spread)
        for G, Am, Bm, C0 in res:
            ref = P.emulated_gemm(Am, Bm, s, alpha, beta, C0)
            assert np.array_equal(G.view(np.int64), ref.view(np.int64)), (s, m, n, k)
        res16 = run_mode(h, "emu", s, m, n, k, alpha, beta, pads=(3, 1, 2), seed=40 + s,
                         spread=spread)
        for (G, _, _, _), (G16, _, _, _) in zip(res, res16):
            assert np.array_equal(G.view(np.int64), G16.view(np.int64))


def test_emulated_zero_rows_and_columns(h):
    A, B, C = _operands(21, 40, 40, 64, 2, (0, 0, 0), 0)
    A[:, :32, 5] = 0.0        # row 5 of A zero in the first chunk
    B[:, 7, :] = 0.0          # column 7 of B zero throughout
    Ad, Bd, Cd = A.cuda(), B.cuda(), C.cuda()
    h.batched_mode("emu", Ad, Bd, Cd, 40, 40, 64, slices=4)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    for i in range(2):
        ref = P.emulated_gemm(_mat(A.numpy()[i], 40), _mat(B.numpy()[i], 64), 4)
        assert np.array_equal(_mat(got[i], 40).view(np.int64), ref.view(np.int64))


def test_emulated_error_falls_with_slices(h):
    errs = []
    for s in range(1, 8):
        res = run_mode(h, "emu", s, 64, 64, 256, seed=31, spread=10, batch=1)
        G, Am, Bm, _ = res[0]
        errs.append(P.relative_errors(G, Am @ Bm)[0])
    for a, b in zip(errs[:5], errs[1:6]):
        assert b < a / 32, errs
    assert errs[6] < 1e-14, errs


def _reduced_bound(mode, Am, Bm, alpha):
    rnd = P.round_fp32 if mode == "fp32" else P.round_bf16
    k = Am.shape[1]
    return (k + 4) * 2.0 ** -23 * abs(alpha) * (np.abs(rnd(Am)) @ np.abs(rnd(Bm)))


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 32), (70, 45, 100), (130, 129, 77),
                                   (5, 200, 31), (17, 3, 500)])
def test_reduced_modes_within_binary32_accumulation(h, mode, m, n, k):
    for alpha, beta, seed in ((1.0, 0.0, 41), (-0.75, 1.5, 42)):
        for G, Am, Bm, C0 in run_mode(h, mode, 0, m, n, k, alpha, beta, seed=seed,
                                      pads=(2, 0, 1)):
            exp = alpha * P.reference_product(Am, Bm, mode) + (beta * C0 if beta else 0.0)
            bound = _reduced_bound(mode, Am, Bm, alpha) + 1e-15 * (np.abs(exp) + abs(beta) * np.abs(C0))
            assert np.all(np.abs(G - exp) <= bound), (mode, m, n, k)


@pytest.mark.parametrize("mode,lo", [("fp32", 1e-9), ("bf16", 1e-4)])
def test_reduced_modes_really_reduce(h, mode, lo):
    G, Am, Bm, _ = run_mode(h, mode, 0, 64, 64, 64, seed=51, batch=1)[0]
    assert P.relative_errors(G, Am @ Bm)[0] > lo


@pytest.mark.parametrize("mode", ["fp32", "bf16", "emu"])
def test_modes_scalar_rules(h, mode):
    s = 4 if mode == "emu" else 0
    A, B, C = _operands(61, 20, 30, 40, 2, (0, 0, 0), 0)
    Ad, Bd = A.cuda(), B.cuda()
    # beta == 1 with alpha == 0: C untouched bit for bit; k == 0: C <- beta C
    Cd = C.cuda()
    h.batched_mode(mode, Ad, Bd, Cd, 20, 30, 40, 0.0, 1.0, slices=s)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu().view(torch.int64), C.view(torch.int64))
    Cd = C.cuda()
    h.batched_mode(mode, Ad, Bd, Cd, 20, 30, 0, 1.0, -2.0, slices=s)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu()[:, :, :20], -2.0 * C[:, :, :20])
    # beta == 0 never reads C (NaN does not propagate)
    Cn = C.clone()
    Cn[:, :, :20] = float("nan")
    Cd = Cn.cuda()
    h.batched_mode(mode, Ad, Bd, Cd, 20, 30, 40, 1.0, 0.0, slices=s)
    torch.cuda.synchronize()
    assert not torch.isnan(Cd.cpu()[:, :, :20]).any()


def test_modes_argument_errors(h):
    A, B, C = _operands(71, 8, 8, 8, 1, (0, 0, 0), 0)
    Ad, Bd, Cd = A.cuda(), B.cuda(), C.cuda()
    with pytest.raises(bgemm.BgemmError) as e:
        h.batched_mode(7, Ad, Bd, Cd, 8, 8, 8)
    assert e.value.status == 1 and e.value.arg == 101
    for bad in (0, 9):
        with pytest.raises(bgemm.BgemmError) as e:
            h.batched_mode("emu", Ad, Bd, Cd, 8, 8, 8, slices=bad)
        assert e.value.status == 1 and e.value.arg == 102
    for ta, tb in (("T", "N"), ("N", "T")):
        with pytest.raises(bgemm.BgemmError) as e:
            h.batched_mode("bf16", Ad, Bd, Cd, 8, 8, 8, transa=ta, transb=tb)
        assert e.value.status == 2
    with pytest.raises(bgemm.BgemmError) as e:
        h.batched_mode("fp32", Ad, Bd, Cd, 8, 8, 8, transa="X")
    assert e.value.status == 1 and e.value.arg == 1
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu().view(torch.int64), C.view(torch.int64))


def test_fp64_mode_is_the_binary64_path(h):
    A, B, C = _operands(81, 33, 31, 65, 2, (0, 0, 0), 0)
    C1, C2 = C.cuda(), C.cuda()
    Ad, Bd = A.cuda(), B.cuda()
    h.batched(Ad, Bd, C1, 33, 31, 65, 0.5, 2.0)
    h.batched_mode("fp64", Ad, Bd, C2, 33, 31, 65, 0.5, 2.0)
    torch.cuda.synchronize()
    assert torch.equal(C1.cpu().view(torch.int64), C2.cpu().view(torch.int64))
