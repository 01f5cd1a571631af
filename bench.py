"""Benchmark of the batched FP64 GEMM hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload config2+vb]

A step is one pass over every part of the workload: the three uniform
batches of 64^3, 256^3 and 512^3 (symmetric) instances through
bg_dgemm_batched and the 100,000-instance variable-size batch through
bg_dgemm_vbatched (device planning + persistent tile-queue kernel).  Inputs
are seeded synthetic matrices already resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_FP64 = 78.6e12      # MI355X published FP64 (vector and matrix), flop/s
PEAK_HBM = 8.0e12        # MI355X published HBM3E bandwidth, bytes/s
METRIC = "batched GEMM GFLOP/s at FP64 accuracy, % roofline; p50/p99 request latency"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "hbm_traffic_config2+vb.md")


def measured_traffic(part: str, workload: str):
    """HBM bytes (read + written) per launch of `part` from the committed
    rocprofv3 counter summary, or None when there is none for this workload or
    the kernels changed since the counters were taken."""
    from paper_2203_09353_amd.profile_summary import kernel_source_hash, load_traffic
    t = load_traffic(TRAFFIC_SUMMARY)
    if not t or t.get("workload") != workload or t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    p = t["parts"].get(part)
    if not p:
        return None
    return {"bytes": round(p["read_bytes"] + p["write_bytes"]), "read": round(p["read_bytes"]),
            "written": round(p["write_bytes"]), "source": "profiles/hbm_traffic_config2+vb.md"}


def part_launch(h, p):
    from paper_2203_09353_amd.workloads import UniformPart
    if isinstance(p, UniformPart):
        pA, pB, pC = p.pointers()
        st = h.dgemm_batched_raw("N", "N", p.m, p.n, p.k, p.alpha, pA.data_ptr(), p.A.shape[-1],
                                 pB.data_ptr(), p.B.shape[-1], p.beta, pC.data_ptr(),
                                 p.C.shape[-1], p.batch)
    else:
        st = h.dgemm_vbatched_raw("N", "N", p.m.data_ptr(), p.n.data_ptr(), p.k.data_ptr(),
                                  p.alpha, p.pA.data_ptr(), p.lda.data_ptr(), p.pB.data_ptr(),
                                  p.ldb.data_ptr(), p.beta, p.pC.data_ptr(), p.ldc.data_ptr(),
                                  p.batch, p.info.data_ptr())
    if st != 0:
        raise RuntimeError("launch of %s failed with status %d" % (p.name, st))


def sampled_parity(h, parts, per_part, seed=11):
    """Runs one step and compares `per_part` seeded instances of every part
    with the CPU oracle (inputs copied to the host before the call)."""
    import numpy as np
    import torch
    import oracle
    from paper_2203_09353_amd import inputs
    from paper_2203_09353_amd.workloads import UniformPart, host_instance

    picks = {}
    for p in parts:
        idx = inputs.permutation(seed, sum(map(ord, p.name)), p.batch)[:per_part].tolist()
        picks[p.name] = [(i, host_instance(p, i)) for i in idx]
    for p in parts:
        part_launch(h, p)
    torch.cuda.synchronize()
    worst = {}
    for p in parts:
        w = 0.0
        for i, (A, B, C0) in picks[p.name]:
            got = host_instance(p, i)[2]
            C = C0.copy()
            if isinstance(p, UniformPart):
                m, n, k = p.m, p.n, p.k
                oracle.gemm("N", "N", m, n, k, p.alpha, A, A.shape[-1], B, B.shape[-1], p.beta,
                            C, C.shape[-1])
            else:
                m, n, k = (int(x[i]) for x in p.sizes_host[:3])
                oracle.gemm("N", "N", m, n, k, p.alpha, A, A.shape[-1], B, B.shape[-1], p.beta,
                            C, C.shape[-1])
            d = np.linalg.norm(got[:n, :m] - C[:n, :m])
            r = np.linalg.norm(C[:n, :m])
            rel = d / r if r else (0.0 if d == 0 else float("inf"))
            w = max(w, rel)
        worst[p.name] = w
    return worst


def cpu_baseline(parts, seconds):
    """Times the CPU oracle, as it stands, on the first instances of every
    part (same mix as the workload), sized for about `seconds` of work."""
    import numpy as np
    import torch
    import oracle
    from paper_2203_09353_amd.workloads import UniformPart

    threads = len(os.sched_getaffinity(0))

    def run(frac):
        flops = 0.0
        t = 0.0
        desc = []
        for p in parts:
            n = max(1, int(p.batch * frac))
            if isinstance(p, UniformPart):
                A = p.A[:n].cpu().numpy(); B = p.B[:n].cpu().numpy(); C = p.C[:n].cpu().numpy()
                t0 = time.perf_counter()
                oracle.gemm_batched("N", "N", p.m, p.n, p.k, p.alpha, A, B, p.beta, C,
                                    nthreads=threads)
                t += time.perf_counter() - t0
                flops += 2.0 * p.m * p.n * p.k * n
            else:
                ms, ns, ks, la, lb, lc = (x[:n].numpy() for x in p.sizes_host)
                As, Bs, Cs = [], [], []
                hosts = [slab[: int(o[n])].cpu().numpy() for slab, o in zip(p.slabs, p.offs)]
                for i in range(n):
                    for lst, host, o, cols, ld in ((As, hosts[0], p.offs[0], ks[i], la[i]),
                                                   (Bs, hosts[1], p.offs[1], ns[i], lb[i]),
                                                   (Cs, hosts[2], p.offs[2], ns[i], lc[i])):
                        a = int(o[i])
                        lst.append(host[a:a + int(cols) * int(ld)].reshape(int(cols), int(ld)))
                t0 = time.perf_counter()
                oracle.gemm_vbatched("N", "N", ms, ns, ks, p.alpha, As, Bs, p.beta, Cs,
                                     ldas=la, ldbs=lb, ldcs=lc, nthreads=threads)
                t += time.perf_counter() - t0
                flops += float((2.0 * ms.astype(np.float64) * ns * ks).sum())
            desc.append("%s:%d/%d" % (p.name, n, p.batch))
        return flops, t, desc

    f0, t0, _ = run(0.001)
    rate = f0 / max(t0, 1e-6)
    total = sum(p.flops for p in parts)
    frac = min(1.0, max(0.001, seconds * rate / total))
    flops, t, desc = run(frac)
    return {"value": round(flops / t / 1e9, 3), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": "first %.2f%% of each part's instances (%s), %.1f s" % (
                100 * frac, ", ".join(desc), t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2+vb")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--check", type=int, default=3, help="sampled parity instances per part")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the batched GEMM instances are independent and "
              "this build has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_09353_amd import bgemm, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    h = bgemm.Handle()
    log("building workload %s" % args.workload)
    t0 = time.perf_counter()
    parts = workloads.build(args.workload, "cuda")
    torch.cuda.synchronize()
    log("built in %.1f s; device memory %.1f GB" % (time.perf_counter() - t0,
                                                     torch.cuda.memory_allocated() / 1e9))

    parity = sampled_parity(h, parts, args.check) if args.check > 0 else {}
    log("sampled parity (max rel Frobenius per part): %s" % parity)

    for _ in range(args.warmup):
        for p in parts:
            part_launch(h, p)
    torch.cuda.synchronize()
    log("warmup done")

    stream = torch.cuda.current_stream()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in parts] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for j, p in enumerate(parts):
            ev[s][j][0].record(stream)
            part_launch(h, p)
            ev[s][j][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("timed %d steps in %.3f s" % (args.steps, elapsed))

    ms_step = elapsed * 1e3 / args.steps
    total_flops = sum(p.flops for p in parts)
    value = total_flops / (ms_step * 1e-3) / 1e9
    part_rows = []
    for j, p in enumerate(parts):
        ms = sum(ev[s][j][0].elapsed_time(ev[s][j][1]) for s in range(args.steps)) / args.steps
        sec = ms * 1e-3
        if hasattr(p, "per_instance_roofline_s"):
            t_roof = p.per_instance_roofline_s(PEAK_FP64, PEAK_HBM)
        else:
            t_roof = max(p.flops / PEAK_FP64, p.bytes / PEAK_HBM)
        ai = p.flops / p.bytes
        part_rows.append({"part": p.name, "instances": p.batch, "ms": round(ms, 4),
                          "gflops": round(p.flops / sec / 1e9, 1),
                          "gbps": round(p.bytes / sec / 1e9, 1),
                          "flop_per_byte": round(ai, 2),
                          "bound": "mfma" if ai >= PEAK_FP64 / PEAK_HBM else "hbm",
                          "roofline_frac": round(t_roof / sec, 4),
                          "parity_max_rel_fro": parity.get(p.name)})
    dom = max(range(len(parts)), key=lambda j: part_rows[j]["ms"])
    dp, dr = parts[dom], part_rows[dom]
    sec = dr["ms"] * 1e-3
    if dr["bound"] == "mfma":
        roof = {"bound": "mfma", "achieved": round(dp.flops / sec / 1e12, 3),
                "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(dp.bytes / sec / 1e9, 1),
                "peak": PEAK_HBM / 1e9, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = measured_traffic(dp.name, args.workload)
    roof["kernel"] = dp.name

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(parts, args.cpu_seconds)

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded counter-based uniform[-1,1); symmetric Q diag Q^T for 512^3)",
           "config": {"workload": args.workload,
                      "parts": ", ".join("%s x%d" % (p.name, p.batch) for p in parts)},
           "roofline": roof, "cpu_baseline": cpu, "parts": part_rows}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
