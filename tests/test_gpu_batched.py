"""GPU parity of the uniform batched path against the CPU oracle, through the
C ABI: every size class, all transposes, padded and tight leading
dimensions, shuffled pointer arrays, integer inputs (bit-exact), the alpha /
beta special cases and the NaN canaries in padding and in C."""
import itertools

import numpy as np
import pytest
import torch

from paper_2203_09353_amd import bgemm, inputs
from tests.parity import check_instance, op_view, oracle_uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def _make(seed, ta, tb, m, n, k, batch, pads, integer, c_nan=False):
    a_rows, a_cols = (k, m) if ta == "T" else (m, k)
    b_rows, b_cols = (n, k) if tb == "T" else (k, n)
    lda = max(1, a_rows + pads[0]); ldb = max(1, b_rows + pads[1]); ldc = max(1, m + pads[2])
    A = inputs.uniform_batch(seed, 0, batch, a_rows, a_cols, lda)
    B = inputs.uniform_batch(seed, 1, batch, b_rows, b_cols, ldb)
    C = inputs.uniform_batch(seed, 2, batch, m, n, ldc)
    if integer:
        A, B, C = (torch.round(X * 32) for X in (A, B, C))
    if c_nan:
        C[:, :, :m] = float("nan")
    return A, B, C, (a_rows, a_cols), (b_rows, b_cols)


def run_case(h, ta, tb, m, n, k, alpha, beta, batch=5, pads=(0, 0, 0), seed=1, integer=False,
             cls=-1, c_nan=False, shuffle=True):
    A, B, C, ash, bsh = _make(seed, ta, tb, m, n, k, batch, pads, integer, c_nan)
    Ad, Bd, Cd = A.cuda(), B.cuda(), C.cuda()
    pA, pB, pC = (bgemm.pointer_array(X) for X in (Ad, Bd, Cd))
    perm = inputs.permutation(seed, 9, batch).cuda() if shuffle else torch.arange(batch).cuda()
    h.set_uniform_class(cls)
    try:
        h.batched(Ad, Bd, Cd, m, n, k, alpha, beta, ta, tb, ptrs=(pA[perm], pB[perm], pC[perm]))
        torch.cuda.synchronize()
    finally:
        h.set_uniform_class(-1)
    got = Cd.cpu().numpy()
    An, Bn, Cn = A.numpy(), B.numpy(), C.numpy()
    ref = oracle_uniform(ta, tb, m, n, k, alpha, An, Bn, beta, Cn)
    # padding rows of C are bit-identical to what was there before the call
    assert np.array_equal(got[:, :, m:].view(np.int64), Cn[:, :, m:].view(np.int64))
    for i in range(batch):
        Aop = op_view(An[i], *ash, ta)
        Bop = op_view(Bn[i], *bsh, tb)
        check_instance(got[i, :, :m].T, ref[i, :, :m].T, Aop, Bop, Cn[i, :, :m].T, alpha, beta,
                       exact=integer, where="inst %d %s%s %dx%dx%d cls %d" % (i, ta, tb, m, n, k, cls))


SHAPES = [(32, 32, 32), (7, 9, 13), (33, 31, 65), (64, 64, 64), (65, 63, 17), (100, 70, 129),
          (130, 129, 77), (1, 200, 3), (257, 5, 31)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("pads", [(0, 0, 0), (3, 1, 5)])
def test_uniform_random(h, m, n, k, ta, tb, pads):
    run_case(h, ta, tb, m, n, k, 1.0, 0.0, pads=pads)
    run_case(h, ta, tb, m, n, k, -0.75, 1.5, pads=pads, seed=2)


@pytest.mark.parametrize("cls", [0, 1, 2])
@pytest.mark.parametrize("m,n,k", [(7, 9, 13), (100, 70, 129), (130, 129, 77), (64, 64, 64)])
def test_every_class_on_every_shape(h, cls, m, n, k):
    for ta, tb in (("N", "N"), ("T", "N"), ("N", "T")):
        run_case(h, ta, tb, m, n, k, 1.0, 0.5, cls=cls, pads=(1, 2, 0), batch=3)


@pytest.mark.parametrize("m,n,k", [(32, 32, 32), (64, 64, 64), (61, 67, 513), (256, 256, 256),
                                   (129, 17, 200)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-2.0, 1.0), (0.5, -1.0)])
def test_uniform_integer_bit_exact(h, m, n, k, alpha, beta):
    for ta, tb in (("N", "N"), ("T", "T")):
        run_case(h, ta, tb, m, n, k, alpha, beta, integer=True, batch=3, pads=(0, 1, 2))


def test_beta_zero_never_reads_C(h):
    # C holds NaN; with beta == 0 the result must be finite
    for cls in (-1, 0, 1, 2):
        run_case(h, "N", "N", 70, 45, 33, 1.0, 0.0, c_nan=True, cls=cls, pads=(2, 2, 3))


def test_alpha_zero_and_k_zero(h):
    m, n, k, batch = 20, 11, 9, 4
    A = torch.full((batch, k, m), float("nan"), dtype=torch.float64, device="cuda")
    B = torch.full((batch, n, k), float("nan"), dtype=torch.float64, device="cuda")
    C0 = inputs.uniform_batch(3, 2, batch, m, n, m + 2)
    C0[0, 0, 0] = -0.0
    Cd = C0.cuda()
    # alpha == 0: A, B not read; C <- 0.5 C
    h.batched(A, B, Cd, m, n, k, 0.0, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(Cd.cpu()[:, :, :m], 0.5 * C0[:, :, :m])
    # alpha == 0, beta == 0: exactly zero even from NaN
    Cd[:, :, :m] = float("nan")
    h.batched(A, B, Cd, m, n, k, 0.0, 0.0)
    torch.cuda.synchronize()
    assert torch.all(Cd.cpu()[:, :, :m] == 0)
    # k == 0 with beta == 1: untouched bit for bit (no launch)
    Cd = C0.cuda()
    h.batched(A, B, Cd, m, n, 0, 3.0, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(Cd.cpu().numpy().view(np.int64), C0.numpy().view(np.int64))


def test_quick_returns_and_errors(h):
    # batch == 0 and m == 0 with NULL arrays: success, no device access
    assert h.dgemm_batched_raw("N", "N", 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 0) == 0
    assert h.dgemm_batched_raw("N", "N", 0, 4, 4, 1.0, None, 1, None, 4, 0.0, None, 1, 7) == 0
    assert h.dgemm_batched_raw("N", "N", 4, 4, 4, 1.0, None, 3, None, 4, 0.0, None, 4, 7) == 1
    assert h.last_invalid_arg() == 8
    assert h.dgemm_batched_raw("N", "Z", 4, 4, 4, 1.0, None, 4, None, 4, 0.0, None, 4, 7) == 1
    assert h.last_invalid_arg() == 2


def test_aliased_gram_product(h):
    # A_i and B_i may alias: C = X^T X
    m, k, batch = 37, 23, 4
    X = inputs.uniform_batch(5, 0, batch, k, m)
    Xd = X.cuda()
    Cd = torch.zeros(batch, m, m, dtype=torch.float64, device="cuda")
    h.batched(Xd, Xd, Cd, m, m, k, 1.0, 0.0, "T", "N")
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    ref = oracle_uniform("T", "N", m, m, k, 1.0, X.numpy(), X.numpy(), 0.0, np.zeros((batch, m, m)))
    for i in range(batch):
        Xi = X.numpy()[i].T
        check_instance(got[i].T, ref[i].T, Xi.T, Xi, np.zeros((m, m)), 1.0, 0.0)


def test_config_1x32_full(h):
    """1000 instances of 32x32x32, alpha = 1, beta = 0, seed 0, C starts as NaN."""
    batch, m = 1000, 32
    A = inputs.uniform_batch(0, 0, batch, m, m)
    B = inputs.uniform_batch(0, 1, batch, m, m)
    C0 = torch.full((batch, m, m), float("nan"), dtype=torch.float64)
    Cd = C0.cuda()
    h.batched(A.cuda(), B.cuda(), Cd, m, m, m, 1.0, 0.0)
    torch.cuda.synchronize()
    got = Cd.cpu().numpy()
    ref = oracle_uniform("N", "N", m, m, m, 1.0, A.numpy(), B.numpy(), 0.0, C0.numpy())
    for i in range(batch):
        check_instance(got[i].T, ref[i].T, A.numpy()[i].T, B.numpy()[i].T, np.zeros((m, m)),
                       1.0, 0.0, where="inst %d" % i)


@pytest.mark.parametrize("m,n,k", [(65, 63, 17), (129, 131, 33), (127, 5, 255), (7, 9, 13),
                                   (130, 66, 64), (257, 129, 47)])
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
def test_pipelined_path_odd_extents_even_ld(h, m, n, k, ta, tb):
    """The 128-tile class loads 16-byte-aligned operands with even leading
    dimensions through its direct-to-LDS pipeline.  Odd extents with even ld
    exercise its edge rules: pairs straddling the last row read ld padding,
    the last column and a partial last k-step go through registers."""
    def even_pad(rows):
        return 1 if rows % 2 else 2
    a_rows = k if ta == "T" else m
    b_rows = n if tb == "T" else k
    pads = (even_pad(a_rows), even_pad(b_rows), even_pad(m))
    run_case(h, ta, tb, m, n, k, 1.0, 0.5, pads=pads, cls=2, batch=3)
    run_case(h, ta, tb, m, n, k, -2.0, 1.0, pads=pads, cls=2, batch=3, integer=True, seed=7)
    # tight even ld where the extent is even
    if a_rows % 2 == 0 and b_rows % 2 == 0 and m % 2 == 0:
        run_case(h, ta, tb, m, n, k, 1.0, 0.0, pads=(0, 0, 0), cls=2, batch=2)


@pytest.mark.parametrize("m,n,k", [(65, 63, 17), (129, 131, 33), (7, 9, 13), (130, 66, 64)])
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
def test_odd_ld_and_unaligned_operands_in_the_pipelined_class(h, m, n, k, ta, tb):
    """Odd leading dimensions and operands that start 8 bytes past a 16-byte
    boundary, in the 128-tile class (whose pipelined path needs 16-byte
    aligned pairs; such tiles must take its other path)."""
    run_case(h, ta, tb, m, n, k, 1.0, 0.5, pads=(1, 3, 1), cls=2, batch=3)
    run_case(h, ta, tb, m, n, k, -2.0, 1.0, pads=(2, 1, 0), cls=2, batch=3, integer=True, seed=9)
    # instance 0 of a stacked batch shifted by one double: every operand
    # pointer is only 8-byte aligned
    A, B, C, ash, bsh = _make(13, ta, tb, m, n, k, 2, (2, 2, 2), False)
    sh = lambda X: torch.cat([torch.zeros(1, dtype=torch.float64), X.reshape(-1)]).cuda()
    fa, fb, fc = sh(A), sh(B), sh(C)
    per = lambda X: X.shape[1] * X.shape[2]
    pA = torch.tensor([fa.data_ptr() + 8 + 8 * i * per(A) for i in range(2)], device="cuda")
    pB = torch.tensor([fb.data_ptr() + 8 + 8 * i * per(B) for i in range(2)], device="cuda")
    pC = torch.tensor([fc.data_ptr() + 8 + 8 * i * per(C) for i in range(2)], device="cuda")
    h.set_uniform_class(2)
    try:
        st = h.dgemm_batched_raw(ta, tb, m, n, k, 0.75, pA.data_ptr(), A.shape[2], pB.data_ptr(),
                                 B.shape[2], -0.5, pC.data_ptr(), C.shape[2], 2)
        torch.cuda.synchronize()
    finally:
        h.set_uniform_class(-1)
    assert st == 0
    got = fc[1:].cpu().numpy().reshape(C.shape)
    ref = oracle_uniform(ta, tb, m, n, k, 0.75, A.numpy(), B.numpy(), -0.5, C.numpy())
    for i in range(2):
        check_instance(got[i, :, :m].T, ref[i, :, :m].T, op_view(A.numpy()[i], *ash, ta),
                       op_view(B.numpy()[i], *bsh, tb), C.numpy()[i, :, :m].T, 0.75, -0.5,
                       where="shifted inst %d" % i)


def test_huge_leading_dimension(h):
    """A leading dimension so large that one 128-row tile spans more than
    2 GB: 64-bit addressing throughout, results as the oracle's."""
    m, n, k, lda = 130, 40, 20, 2_200_000          # A stored k x m ('T'), 2.3 GB
    A = torch.full((1, m, lda), float("nan"), dtype=torch.float64, device="cuda")
    Ac = inputs.uniform_batch(71, 0, 1, k, m, k)    # compact copy for the oracle
    A[:, :, :k] = Ac.cuda()
    B = inputs.uniform_batch(71, 1, 1, k, n, k)
    C = inputs.uniform_batch(71, 2, 1, m, n, m)
    Cd = C.cuda()
    h.set_uniform_class(2)
    try:
        h.batched(A, B.cuda(), Cd, m, n, k, 1.0, 0.5, "T", "N")
        torch.cuda.synchronize()
    finally:
        h.set_uniform_class(-1)
    del A
    got = Cd.cpu().numpy()
    ref = oracle_uniform("T", "N", m, n, k, 1.0, Ac.numpy(), B.numpy(), 0.5, C.numpy())
    check_instance(got[0, :, :m].T, ref[0, :, :m].T, op_view(Ac.numpy()[0], k, m, "T"),
                   op_view(B.numpy()[0], k, n, "N"), C.numpy()[0, :, :m].T, 1.0, 0.5,
                   where="huge lda")
