"""The variable-size entry point that allocates nothing
(bg_dgemm_vbatched_noalloc, planning buffers in the library's static device
array), called through the C ABI: two calls in a row, the second with a
smaller batch, each bit-identical to bg_dgemm_vbatched on the same inputs and
within the oracle's bounds; invalid instances reported in d_info and left
untouched; host argument errors and batches beyond the array's capacity
refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09353_amd import bgemm, inputs
from tests.parity import check_instance, op_view

pytestmark = pytest.mark.gpu


def _batch(seed, count, bad=()):
    ms, ns, ks = (inputs.log_uniform_sizes(seed, s, count).tolist() for s in range(3))
    for i in bad:
        ms[i] = -1          # an invalid instance: d_info -3, C untouched
    rows = lambda x: max(x, 0)
    As = inputs.uniform_ragged(seed, 0, [rows(m) for m in ms], ks)
    Bs = inputs.uniform_ragged(seed, 1, ks, ns)
    Cs = inputs.uniform_ragged(seed, 2, [rows(m) for m in ms], ns)
    fix = lambda L: [x if x.numel() else torch.zeros(1, 1, dtype=torch.float64) for x in L]
    return ms, ns, ks, fix(As), fix(Bs), fix(Cs)


def _device_args(ms, ns, ks, As, Bs, Cs):
    dev = torch.device("cuda", torch.cuda.current_device())
    iv = lambda x: torch.tensor(list(x), dtype=torch.int32, device=dev)
    Ad = [a.cuda() for a in As]; Bd = [b.cuda() for b in Bs]; Cd = [c.cuda() for c in Cs]
    t = dict(m=iv(ms), n=iv(ns), k=iv(ks), lda=iv([a.shape[-1] for a in As]),
             ldb=iv([b.shape[-1] for b in Bs]), ldc=iv([c.shape[-1] for c in Cs]),
             pA=bgemm.pointer_array(Ad), pB=bgemm.pointer_array(Bd), pC=bgemm.pointer_array(Cd),
             info=torch.full((len(ms),), 7, dtype=torch.int32, device=dev))
    return Ad, Bd, Cd, t


def _noalloc(t, batch, alpha, beta, transa="N"):
    return bgemm.dgemm_vbatched_noalloc_raw(
        transa, "N", t["m"].data_ptr(), t["n"].data_ptr(), t["k"].data_ptr(), alpha,
        t["pA"].data_ptr(), t["lda"].data_ptr(), t["pB"].data_ptr(), t["ldb"].data_ptr(), beta,
        t["pC"].data_ptr(), t["ldc"].data_ptr(), batch, t["info"].data_ptr())


def _one_call(h, seed, count, bad, alpha, beta):
    ms, ns, ks, As, Bs, Cs = _batch(seed, count, bad)
    # the handle's entry point on its own copy of C
    C_ref_dev = [c.cuda() for c in Cs]
    info_h = h.vbatched([a.cuda() for a in As], [b.cuda() for b in Bs], C_ref_dev, ms, ns, ks,
                        alpha, beta)
    _, _, Cd, t = _device_args(ms, ns, ks, As, Bs, Cs)
    st, bad_arg = _noalloc(t, count, alpha, beta)
    assert (st, bad_arg) == (0, 0)
    torch.cuda.synchronize()
    assert torch.equal(t["info"], info_h)
    Cref = [c.numpy().copy() for c in Cs]
    oinfo = oracle.gemm_vbatched("N", "N", ms, ns, ks, alpha, [a.numpy() for a in As],
                                 [b.numpy() for b in Bs], beta, Cref)
    assert np.array_equal(t["info"].cpu().numpy(), oinfo)
    for i in range(count):
        got = Cd[i].cpu().numpy()
        assert np.array_equal(got.view(np.int64), C_ref_dev[i].cpu().numpy().view(np.int64)), i
        if oinfo[i] != 0:
            assert np.array_equal(got.view(np.int64), Cs[i].numpy().view(np.int64)), i
            continue
        m, n, k = ms[i], ns[i], ks[i]
        check_instance(got[:n, :m].T, Cref[i][:n, :m].T, op_view(As[i].numpy(), m, k, "N"),
                       op_view(Bs[i].numpy(), k, n, "N"), Cs[i].numpy()[:n, :m].T, alpha, beta,
                       where="inst %d (%d,%d,%d)" % (i, m, n, k))


def test_noalloc_two_calls_match_handle_path():
    h = bgemm.Handle()
    try:
        print("[no-alloc] call 1: 1200 instances", flush=True)
        _one_call(h, 61, 1200, bad=(5, 600), alpha=1.0, beta=0.5)
        print("[no-alloc] call 2: 150 instances", flush=True)
        _one_call(h, 62, 150, bad=(3,), alpha=-0.75, beta=0.0)
    finally:
        h.close()


def test_noalloc_refusals_enqueue_nothing():
    ms, ns, ks, As, Bs, Cs = _batch(63, 20)
    _, _, Cd, t = _device_args(ms, ns, ks, As, Bs, Cs)
    st, bad = _noalloc(t, 20, 1.0, 0.5, transa="X")
    assert (st, bad) == (1, 1)
    st, bad = _noalloc(t, -1, 1.0, 0.5)
    assert (st, bad) == (1, 14)
    cap = bgemm.lib().bg_noalloc_max_batch()
    assert 600_000 < cap < 1_000_000
    # beyond the array's capacity: refused on the host before any launch, so
    # the (short) device arrays are never read
    st, bad = _noalloc(t, cap + 1, 1.0, 0.5)
    assert (st, bad) == (6, 0)
    torch.cuda.synchronize()
    assert int((t["info"] != 7).sum()) == 0
    for i in range(20):
        assert torch.equal(Cd[i].cpu().view(torch.int64), Cs[i].view(torch.int64))
