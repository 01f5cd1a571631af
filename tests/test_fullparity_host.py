"""The every-instance parity helpers used by the full-size GPU tests, run on
the CPU: a correct result (the oracle's own) passes, a result with one
perturbed element in one instance is caught, and the spectral identities of
the symmetric part hold on the oracle's products."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_09353_amd import workloads
from tests import fullparity


def _oracle_uniform(p):
    C = p.C.numpy()
    oracle.gemm_batched("N", "N", p.m, p.n, p.k, p.alpha, p.A.numpy(), p.B.numpy(), p.beta, C)


def _oracle_vb(p):
    ms, ns, ks, la, lb, lc = (x.numpy() for x in p.sizes_host)
    v = lambda slab, o, i, cols, ld: slab.numpy()[o[i]:o[i] + cols * ld].reshape(cols, ld)
    oA, oB, oC = (o.numpy() for o in p.offs)
    n = p.batch
    As = [v(p.slabs[0], oA, i, ks[i], la[i]) for i in range(n)]
    Bs = [v(p.slabs[1], oB, i, ns[i], lb[i]) for i in range(n)]
    Cs = [v(p.slabs[2], oC, i, ns[i], lc[i]) for i in range(n)]
    oracle.gemm_vbatched("N", "N", ms, ns, ks, p.alpha, As, Bs, p.beta, Cs, ldas=la, ldbs=lb,
                         ldcs=lc)
    p.info.zero_()


def test_uniform_helper_accepts_oracle_and_catches_one_bad_element():
    p = workloads.build("u64", "cpu", scale=0.0002)[0]
    C0 = p.C.clone()
    assert fullparity.every_instance_uniform(lambda: _oracle_uniform(p), p, 1 << 20) < 1e-15
    p.C.copy_(C0)

    def bad():
        _oracle_uniform(p)
        p.C[p.batch - 1, 3, 5] *= 1.0 + 1e-12
    with pytest.raises(AssertionError):
        fullparity.every_instance_uniform(bad, p, 1 << 20)


@pytest.mark.parametrize("pad8", [False, True])
def test_vb_helper_accepts_oracle_and_catches_one_bad_element(pad8):
    p = workloads.build("vb8" if pad8 else "vb", "cpu", scale=0.0005)[0]
    slab0 = p.slabs[2].clone()
    assert fullparity.every_instance_vb(lambda: _oracle_vb(p), p, 1 << 22) < 1e-15
    p.slabs[2].copy_(slab0)

    def bad():
        _oracle_vb(p)
        o = int(p.offs[2][p.batch - 1])
        p.slabs[2][o] += 1e-9
    with pytest.raises(AssertionError):
        fullparity.every_instance_vb(bad, p, 1 << 22)


def test_symmetric_identities_hold_on_oracle_products():
    p = workloads.build("s512", "cpu", scale=0.0202)[0]     # 101 instances: 0 and 100 share Q
    picks = [i for i in range(p.batch) if i % 100 == 0]
    C0 = {i: p.C[i].numpy().copy() for i in picks}
    _oracle_uniform(p)
    assert fullparity.symmetric_identities(p, C0) == len(picks) == 2
    # a product of a wrong instance pair fails the identities
    p.C[100].copy_(torch.from_numpy(C0[100]) + (p.C[0] - torch.from_numpy(C0[0])))
    with pytest.raises(AssertionError):
        fullparity.symmetric_identities(p, {100: C0[100]})
