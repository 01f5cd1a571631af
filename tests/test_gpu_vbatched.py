"""GPU parity of the variable-size batched path (persistent tile-queue kernel)
against the CPU oracle, through the C ABI: log-uniform sizes 2^j - 1 .. 2^j + 1,
tight and padded leading dimensions, transposes, zero sizes, invalid instances
(d_info and untouched C), integer inputs (bit-exact), and results that do not
depend on the rest of the batch."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09353_amd import bgemm, inputs
from tests.parity import check_instance, op_view

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def make_batch(seed, ms, ns, ks, ta, tb, pad8, integer=False):
    a_rows = [k if ta == "T" else m for m, k in zip(ms, ks)]
    a_cols = [m if ta == "T" else k for m, k in zip(ms, ks)]
    b_rows = [n if tb == "T" else k for n, k in zip(ns, ks)]
    b_cols = [k if tb == "T" else n for n, k in zip(ns, ks)]
    ld = (lambda r: inputs.round_up(max(r, 1), 8)) if pad8 else (lambda r: max(r, 1))
    ldas = [ld(r) for r in a_rows]; ldbs = [ld(r) for r in b_rows]; ldcs = [ld(max(m, 0)) for m in ms]
    As = inputs.uniform_ragged(seed, 0, [max(r, 0) for r in a_rows], [max(c, 0) for c in a_cols], ldas)
    Bs = inputs.uniform_ragged(seed, 1, [max(r, 0) for r in b_rows], [max(c, 0) for c in b_cols], ldbs)
    Cs = inputs.uniform_ragged(seed, 2, [max(m, 0) for m in ms], [max(n, 0) for n in ns], ldcs)
    if integer:
        As, Bs, Cs = ([torch.round(x * 32) for x in L] for L in (As, Bs, Cs))
    # every instance owns at least one element so that its pointer is distinct
    fix = lambda L: [x if x.numel() else torch.zeros(1, 1, dtype=torch.float64) for x in L]
    return fix(As), fix(Bs), fix(Cs), ldas, ldbs, ldcs, (a_rows, a_cols, b_rows, b_cols)


def run_vb(h, ms, ns, ks, alpha, beta, ta="N", tb="N", pad8=False, seed=3, integer=False,
           ldas=None, ldcs=None, shuffle=True):
    batch = len(ms)
    As, Bs, Cs, la, lb, lc, shp = make_batch(seed, ms, ns, ks, ta, tb, pad8, integer)
    la = la if ldas is None else ldas
    lc = lc if ldcs is None else ldcs
    Ad = [x.cuda() for x in As]; Bd = [x.cuda() for x in Bs]; Cd = [x.cuda() for x in Cs]
    order = inputs.permutation(seed, 7, batch).tolist() if shuffle else list(range(batch))
    # present the instances to the library in shuffled order
    sel = lambda L: [L[i] for i in order]
    info = h.vbatched(sel(Ad), sel(Bd), sel(Cd), sel(ms), sel(ns), sel(ks), alpha, beta, ta, tb,
                      ldas=sel(la), ldbs=sel(lb), ldcs=sel(lc))
    torch.cuda.synchronize()
    info_sorted = np.empty(batch, dtype=np.int32)
    info_sorted[order] = info.cpu().numpy()
    got = [c.cpu().numpy() for c in Cd]
    Cref = [c.numpy().copy() for c in Cs]
    oinfo = oracle.gemm_vbatched(ta, tb, ms, ns, ks, alpha, [a.numpy() for a in As],
                                 [b.numpy() for b in Bs], beta, Cref, ldas=la, ldbs=lb, ldcs=lc)
    assert np.array_equal(info_sorted, oinfo)
    a_rows, a_cols, b_rows, b_cols = shp
    for i in range(batch):
        m, n = ms[i], ns[i]
        C0 = Cs[i].numpy()
        if oinfo[i] != 0 or m <= 0 or n <= 0:
            assert np.array_equal(got[i].view(np.int64), C0.view(np.int64)), "inst %d touched" % i
            continue
        # padding untouched
        assert np.array_equal(got[i][:, m:].view(np.int64), C0[:, m:].view(np.int64))
        Aop = op_view(As[i].numpy(), a_rows[i], a_cols[i], ta) if ks[i] > 0 else np.zeros((m, 0))
        Bop = op_view(Bs[i].numpy(), b_rows[i], b_cols[i], tb) if ks[i] > 0 else np.zeros((0, n))
        check_instance(got[i][:n, :m].T, Cref[i][:n, :m].T, Aop, Bop, C0[:n, :m].T, alpha, beta,
                       exact=integer, where="inst %d (%d,%d,%d) %s%s" % (i, m, n, ks[i], ta, tb))
    return got


def sizes(seed, count):
    return [inputs.log_uniform_sizes(seed, s, count).tolist() for s in range(3)]


@pytest.mark.parametrize("pad8", [False, True])
def test_vbatched_log_uniform(h, pad8):
    ms, ns, ks = sizes(21, 300)
    run_vb(h, ms, ns, ks, 1.0, 0.5, pad8=pad8)


@pytest.mark.parametrize("ta,tb", [("T", "N"), ("N", "T"), ("T", "T")])
def test_vbatched_transposes(h, ta, tb):
    ms, ns, ks = sizes(22, 120)
    run_vb(h, ms, ns, ks, -1.25, 2.0, ta=ta, tb=tb, pad8=True)


def test_vbatched_integer_exact(h):
    ms, ns, ks = sizes(23, 150)
    run_vb(h, ms, ns, ks, 2.0, -1.0, integer=True)
    run_vb(h, ms, ns, ks, 1.0, 0.0, integer=True, ta="T", tb="T", pad8=True)


def test_vbatched_degenerate_and_invalid(h):
    ms = [0, 5, 7, 9, -1, 4, 16, 3, 65, 1]
    ns = [3, 0, 7, 9, 2, -2, 16, 3, 1, 1]
    ks = [4, 4, 0, 9, 2, 2, -3, 3, 17, 1]
    # instance 7: ldc 2 < m 3 (invalid, -13); instance 9: lda 0 (invalid, -8)
    As, Bs, Cs, la, lb, lc, _ = make_batch(4, ms, ns, ks, "N", "N", False)
    lc = list(lc); la = list(la)
    lc[7] = 2; la[9] = 0
    run_vb(h, ms, ns, ks, 1.0, 0.5, seed=4, ldas=la, ldcs=lc)
    # beta == 1 and k == 0: no-op; beta == 0 with k == 0: exact zeros
    run_vb(h, ms, ns, ks, 1.0, 1.0, seed=4, ldas=la, ldcs=lc)
    run_vb(h, ms, ns, ks, 1.0, 0.0, seed=4, ldas=la, ldcs=lc)


def test_vbatched_alpha_zero(h):
    ms, ns, ks = sizes(24, 40)
    run_vb(h, ms, ns, ks, 0.0, 0.5)


def test_vbatched_result_independent_of_batch_mix(h):
    """Each instance's result is bit-identical alone and inside a larger mix."""
    ms, ns, ks = sizes(25, 60)
    As, Bs, Cs, la, lb, lc, _ = make_batch(5, ms, ns, ks, "N", "N", True)
    Ad = [x.cuda() for x in As]; Bd = [x.cuda() for x in Bs]
    Cmix = [x.cuda() for x in Cs]
    h.vbatched(Ad, Bd, Cmix, ms, ns, ks, 1.0, 0.5, ldas=la, ldbs=lb, ldcs=lc)
    for i in (0, 7, 33, 59):
        Calone = [Cs[i].cuda()]
        h.vbatched([Ad[i]], [Bd[i]], Calone, [ms[i]], [ns[i]], [ks[i]], 1.0, 0.5,
                   ldas=[la[i]], ldbs=[lb[i]], ldcs=[lc[i]])
        torch.cuda.synchronize()
        assert torch.equal(Calone[0].view(torch.int64), Cmix[i].view(torch.int64)), i


def test_vbatched_equals_batched_bitwise(h):
    """Equal sizes through the variable-size path give the same bits as the
    uniform path under every size class: the per-element summation order
    depends only on k."""
    m, n, k, batch = 70, 45, 100, 12
    A = inputs.uniform_batch(6, 0, batch, m, k).cuda()
    B = inputs.uniform_batch(6, 1, batch, k, n).cuda()
    C0 = inputs.uniform_batch(6, 2, batch, m, n).cuda()
    outs = []
    for cls in (0, 1, 2):
        C = C0.clone()
        h.set_uniform_class(cls)
        h.batched(A, B, C, m, n, k, 1.0, 0.5)
        h.set_uniform_class(-1)
        outs.append(C)
    Cv = C0.clone()
    h.vbatched(list(A), list(B), list(Cv), [m] * batch, [n] * batch, [k] * batch, 1.0, 0.5)
    torch.cuda.synchronize()
    for C in outs[1:] + [Cv]:
        assert torch.equal(C.view(torch.int64), outs[0].view(torch.int64))


def test_vbatched_errors(h):
    assert h.dgemm_vbatched_raw("N", "N", None, None, None, 1.0, None, None, None, None, 0.0,
                                None, None, 0, None) == 0
    assert h.dgemm_vbatched_raw("Q", "N", None, None, None, 1.0, None, None, None, None, 0.0,
                                None, None, 3, None) == 1
    assert h.last_invalid_arg() == 1
    assert h.dgemm_vbatched_raw("N", "N", None, None, None, 1.0, None, None, None, None, 0.0,
                                None, None, -1, None) == 1
    assert h.last_invalid_arg() == 14
    assert h.dgemm_vbatched_raw("N", "N", None, None, None, 1.0, None, None, None, None, 0.0,
                                None, None, 3, None) == 1
    assert h.last_invalid_arg() == 3


def test_vbatched_without_tile_map_and_workspace_too_small():
    """A workspace of exactly bg_workspace_bytes_needed(batch) bytes leaves no
    room for the tile -> instance map, so the executor finds each tile's
    instance by binary search over the per-class prefix sums.  The results
    must match the oracle and be bit-identical to the map path; one byte less
    must be refused with BG_STATUS_WORKSPACE_TOO_SMALL and leave C untouched."""
    batch = 700
    ms, ns, ks = sizes(26, batch)
    As, Bs, Cs, la, lb, lc, shp = make_batch(8, ms, ns, ks, "N", "N", False)
    Ad = [x.cuda() for x in As]; Bd = [x.cuda() for x in Bs]
    C_map = [x.cuda() for x in Cs]
    with_map = bgemm.Handle()
    info = with_map.vbatched(Ad, Bd, C_map, ms, ns, ks, 1.0, 0.5, ldas=la, ldbs=lb, ldcs=lc)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(info)) == 0
    need = with_map._L.bg_workspace_bytes_needed(batch)
    assert need > 0
    no_map = bgemm.Handle(workspace_bytes=need)
    try:
        C_find = [x.cuda() for x in Cs]
        info = no_map.vbatched(Ad, Bd, C_find, ms, ns, ks, 1.0, 0.5, ldas=la, ldbs=lb, ldcs=lc)
        torch.cuda.synchronize()
        assert int(torch.count_nonzero(info)) == 0
        for i in range(batch):
            assert torch.equal(C_find[i].view(torch.int64), C_map[i].view(torch.int64)), i
        Cref = [c.numpy().copy() for c in Cs]
        oracle.gemm_vbatched("N", "N", ms, ns, ks, 1.0, [a.numpy() for a in As],
                             [b.numpy() for b in Bs], 0.5, Cref, ldas=la, ldbs=lb, ldcs=lc)
        a_rows, a_cols, b_rows, b_cols = shp
        for i in range(batch):
            m, n, k = ms[i], ns[i], ks[i]
            got = C_find[i].cpu().numpy()
            check_instance(got[:n, :m].T, Cref[i][:n, :m].T,
                           op_view(As[i].numpy(), a_rows[i], a_cols[i], "N"),
                           op_view(Bs[i].numpy(), b_rows[i], b_cols[i], "N"),
                           Cs[i].numpy()[:n, :m].T, 1.0, 0.5, where="inst %d" % i)
        # one byte short: refused before any launch
        no_map.set_workspace(need - 1)
        C_short = [x.cuda() for x in Cs]
        with pytest.raises(bgemm.BgemmError) as e:
            no_map.vbatched(Ad, Bd, C_short, ms, ns, ks, 1.0, 0.5, ldas=la, ldbs=lb, ldcs=lc)
        assert e.value.status == 6          # BG_STATUS_WORKSPACE_TOO_SMALL
        torch.cuda.synchronize()
        for i in (0, batch // 2, batch - 1):
            assert torch.equal(C_short[i].cpu().view(torch.int64), Cs[i].view(torch.int64))
    finally:
        no_map.close()
        with_map.close()
