"""Every-instance parity of a full-size workload part: the part is run once on
the GPU in the benchmark's launch configuration, then every instance is
compared with the CPU oracle, copying inputs and results to the host in
chunks of about ``chunk_bytes``.

Per instance (binary64 paths): ||C_gpu - C_ref||_F <= 1e-13 ||C_ref||_F and,
elementwise, |C_gpu - C_ref| <= (2 gamma_k + 4u)(|alpha||A||B| + |beta||C0|)
(both results obey Higham's bound |fl(AB) - AB| <= gamma_k |A||B|, Accuracy
and Stability of Numerical Algorithms, Section 3.5, plus the roundings of the
alpha/beta update), all entries finite, and the ld padding of C untouched."""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
from tests.colmajor import U, gamma

REL_FRO = 1e-13
TINY = 1e-300


def _sync(t):
    if t.is_cuda:
        torch.cuda.synchronize()


def _threads():
    return len(os.sched_getaffinity(0))


def _check_chunk_uniform(G, R, A, B, C0, alpha, beta, k, first):
    """Stacked storage arrays (cnt, cols, ld) with ld == rows."""
    cnt = G.shape[0]
    assert np.isfinite(G).all(), "non-finite result in instances %d.." % first
    d = np.linalg.norm((G - R).reshape(cnt, -1), axis=1)
    r = np.linalg.norm(R.reshape(cnt, -1), axis=1)
    bad = ~((d <= REL_FRO * r) | ((r == 0) & (d == 0)))
    assert not bad.any(), "instance %d: rel Frobenius %.3e" % (
        first + int(np.argmax(bad)), float((d / np.where(r > 0, r, 1))[bad][0]))
    # storage of C is C^T = B^T A^T: (n x k) @ (k x m) on the stored arrays
    mag = abs(alpha) * np.matmul(np.abs(B), np.abs(A))
    if beta != 0:
        mag += abs(beta) * np.abs(C0)
    over = np.abs(G - R) > (2 * gamma(max(k, 1)) + 4 * U) * mag + TINY
    assert not over.any(), "instance %d: %d elements above the componentwise bound" % (
        first + int(np.argwhere(over)[0][0]), int(over.sum()))
    return float((d / np.where(r > 0, r, 1)).max())


def every_instance_uniform(launch, p, chunk_bytes=1 << 31):
    """`launch()` runs the part once; p is a workloads.UniformPart (NN,
    tight leading dimensions).  Returns the worst relative Frobenius error."""
    C0 = p.C.clone()
    launch()
    _sync(p.C)
    per = 8 * (p.m * p.k + p.k * p.n + 3 * p.m * p.n)
    chunk = max(1, chunk_bytes // per)
    worst = 0.0
    for s in range(0, p.batch, chunk):
        e = min(p.batch, s + chunk)
        A = p.A[s:e].cpu().numpy()
        B = p.B[s:e].cpu().numpy()
        C0h = C0[s:e].cpu().numpy()
        G = p.C[s:e].cpu().numpy()
        R = C0h.copy()
        oracle.gemm_batched("N", "N", p.m, p.n, p.k, p.alpha, A, B, p.beta, R,
                            nthreads=_threads())
        worst = max(worst, _check_chunk_uniform(G, R, A, B, C0h, p.alpha, p.beta, p.k, s))
    del C0
    return worst


def symmetric_identities(p, C0_host: dict, seed=3):
    """Pin P7 on the instances of a symmetric part whose A and B share their
    orthogonal basis (A = Q Da Q^T, B = Q Db Q^T, so A B = Q Da Db Q^T):
    tr(C - C0) = sum da db and ||C - C0||_F^2 = sum (da db)^2 (alpha = beta =
    1).  C0_host maps instance -> its C before the call."""
    from paper_2203_09353_amd import inputs
    qa, qb = p.sym
    n = p.m
    checked = 0
    for i in C0_host:
        assert int(qa[i]) == int(qb[i])
        da = inputs.uniform_flat(seed, 0, i * n, n).numpy()
        db = inputs.uniform_flat(seed, 1, i * n, n).numpy()
        P = (p.C[i].cpu().numpy() - C0_host[i]).T
        lam = da * db
        tr, fro = np.trace(P), np.linalg.norm(P)
        assert abs(tr - lam.sum()) <= 1e-13 * np.abs(lam).sum(), (i, tr, lam.sum())
        assert abs(fro - np.linalg.norm(lam)) <= 1e-13 * np.linalg.norm(lam), (i, fro)
        checked += 1
    return checked


def every_instance_vb(launch, p, chunk_bytes=1 << 31):
    """`launch()` runs the part once; p is a workloads.VbPart (NN).  Checks
    every instance (natural order) and the ld padding of C.  Returns the
    worst relative Frobenius error."""
    C0_slab = p.slabs[2].clone()
    launch()
    _sync(C0_slab)
    assert int(torch.count_nonzero(p.info)) == 0
    ms, ns, ks, la, lb, lc = (x.numpy() for x in p.sizes_host)
    oA, oB, oC = (o.numpy() for o in p.offs)
    worst = 0.0
    s = 0
    while s < p.batch:
        # a run of instances whose data fits the chunk
        e = s + 1
        while e < p.batch and 8 * ((oA[e + 1] - oA[s]) + (oB[e + 1] - oB[s]) +
                                   3 * (oC[e + 1] - oC[s])) <= chunk_bytes:
            e += 1
        hA = p.slabs[0][oA[s]:oA[e]].cpu().numpy()
        hB = p.slabs[1][oB[s]:oB[e]].cpu().numpy()
        hC0 = C0_slab[oC[s]:oC[e]].cpu().numpy()
        hG = p.slabs[2][oC[s]:oC[e]].cpu().numpy()
        hR = hC0.copy()
        view = lambda h, o, i, cols, ld: h[o[i] - o[s]:o[i] - o[s] + cols * ld].reshape(cols, ld)
        idx = range(s, e)
        As = [view(hA, oA, i, ks[i], la[i]) for i in idx]
        Bs = [view(hB, oB, i, ns[i], lb[i]) for i in idx]
        Rs = [view(hR, oC, i, ns[i], lc[i]) for i in idx]
        oracle.gemm_vbatched("N", "N", ms[s:e], ns[s:e], ks[s:e], p.alpha, As, Bs, p.beta, Rs,
                             ldas=la[s:e], ldbs=lb[s:e], ldcs=lc[s:e], nthreads=_threads())
        for j, i in enumerate(idx):
            m, n, k = int(ms[i]), int(ns[i]), int(ks[i])
            G = view(hG, oC, i, n, lc[i])
            C0 = view(hC0, oC, i, n, lc[i])
            R = Rs[j]
            if lc[i] > m:   # padding rows of C keep their bits
                assert np.array_equal(G[:, m:].view(np.int64), C0[:, m:].view(np.int64)), i
            g, r, c0 = G[:, :m], R[:, :m], C0[:, :m]
            assert np.isfinite(g).all(), "instance %d: non-finite result" % i
            dn, rn = np.linalg.norm(g - r), np.linalg.norm(r)
            assert dn <= REL_FRO * rn or (rn == 0 and dn == 0), \
                "instance %d (%d,%d,%d): rel Frobenius %.3e" % (i, m, n, k, dn / rn)
            worst = max(worst, dn / rn if rn else 0.0)
            mag = abs(p.alpha) * (np.abs(Bs[j][:, :k]) @ np.abs(As[j][:, :m]))
            if p.beta != 0:
                mag += abs(p.beta) * np.abs(c0)
            over = np.abs(g - r) > (2 * gamma(max(k, 1)) + 4 * U) * mag + TINY
            assert not over.any(), "instance %d (%d,%d,%d): %d elements above the bound" % (
                i, m, n, k, int(over.sum()))
        s = e
    del C0_slab
    return worst
