"""Where the variable-size batch spends its time: the 100,000-instance
workload (sizes 2^j - 1, 2^j, 2^j + 1 for j = 3..9, independently for m, n
and k) is cut into sub-batches by k, by max(m, n) and by size family, each
launched alone through bg_dgemm_vbatched; every line gives the sub-batch's
event-timed milliseconds, its roofline time (sum over instances of
max(flops / 78.6 TFLOP/s, bytes / 8 TB/s)) and the fraction.

    python -m paper_2203_09353_amd.vb_breakdown [--reps 5]
"""
from __future__ import annotations

import argparse
import json

import torch

from . import bgemm, workloads

PEAK_FLOPS, PEAK_BW = 78.6e12, 8e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    p = workloads.build("vb")[0]
    h = bgemm.Handle(workspace_bytes=256 << 20)
    torch.cuda.synchronize()
    hm, hn, hk = p.m.cpu().double(), p.n.cpu().double(), p.k.cpu().double()

    def run(name, idx):
        ii = idx.cuda()
        sub = [x.index_select(0, ii).contiguous()
               for x in (p.m, p.n, p.k, p.lda, p.ldb, p.ldc, p.pA, p.pB, p.pC)]
        info = torch.empty(len(idx), dtype=torch.int32, device="cuda")

        def go():
            st = h.dgemm_vbatched_raw("N", "N", sub[0].data_ptr(), sub[1].data_ptr(),
                                      sub[2].data_ptr(), p.alpha, sub[6].data_ptr(),
                                      sub[3].data_ptr(), sub[7].data_ptr(), sub[4].data_ptr(),
                                      p.beta, sub[8].data_ptr(), sub[5].data_ptr(), len(idx),
                                      info.data_ptr())
            if st != 0:
                raise RuntimeError("bg_dgemm_vbatched failed with status %d" % st)

        go()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.reps):
            go()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.reps
        m, n, k = hm[idx], hn[idx], hk[idx]
        c_rw = 2 if p.beta != 0 else 1
        f = 2 * m * n * k
        b = 8 * (m * k + k * n + c_rw * m * n) + 48
        roof = float(torch.maximum(f / PEAK_FLOPS, b / PEAK_BW).sum()) * 1e3
        print(json.dumps({"subset": name, "instances": int(len(idx)), "ms": round(ms, 3),
                          "roofline_ms": round(roof, 3), "fraction": round(roof / ms, 3)}),
              flush=True)

    run("all", torch.arange(p.batch))
    buckets = [(2 ** j - 1, 2 ** j + 1) for j in range(3, 10)]
    for lo, hi in buckets:
        run("k %d..%d" % (lo, hi), torch.nonzero((hk >= lo) & (hk <= hi)).flatten())
    mn = torch.maximum(hm, hn)
    for lo, hi in buckets:
        run("max(m,n) %d..%d" % (lo, hi), torch.nonzero((mn >= lo) & (mn <= hi)).flatten())
    ispow = lambda x: x == 2 ** torch.round(torch.log2(x))
    plus1 = lambda x: ispow(x - 1)
    for name, sel in (("m or n = 2^j + 1", plus1(hm) | plus1(hn)),
                      ("m and n powers of two", ispow(hm) & ispow(hn)),
                      ("m or n = 2^j - 1, none 2^j + 1",
                       (ispow(hm + 1) | ispow(hn + 1)) & ~(plus1(hm) | plus1(hn)))):
        run(name, torch.nonzero(sel).flatten())
    h.close()


if __name__ == "__main__":
    main()
