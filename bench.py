"""Benchmark of the batched FP64 GEMM hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload config2+vb]
    python bench.py --workload config4 [--modes fp64,fp32,bf16,emu3,emu6,emu7,f32emu3,f32emu6,i8emu6,...]
    python bench.py --workload config5 [--rates 1000,5000,20000,50000] [--duration 2]
    python bench.py --workload gram15|gram21 [--steps K]
    python bench.py --workload gate21 [--steps K]
    python bench.py --workload config1|vb8 [--cold]
    python bench.py --workload ksweep [--steps K]

A step is one pass over every part of the workload: the three uniform
batches of 64^3, 256^3 and 512^3 (symmetric) instances through
bg_dgemm_batched and the 100,000-instance variable-size batch through
bg_dgemm_vbatched (device planning + persistent tile-queue kernel).  Inputs
are seeded synthetic matrices already resident in HBM.  Prints one JSON line.

``--workload config4`` times the precision modes of bg_gemm_batched_mode on
20,000 wide-exponent 256^3 instances instead: per mode the time, the
binary64-equivalent GFLOP/s and the error on sampled instances against the
binary64 oracle and a compensated (Dot2) reference, judged on at least 32
sampled instances; ``value`` is the fastest mode that reaches binary64
accuracy (relative Frobenius error <= 1e-13).  The binary64 path is always
timed; if no mode meets the rule the run ends with status 3 and no line.

``--workload config5`` drives the request loop (include/bgserve.h): 64
clients with states of 2^k x 2^k (k uniform in 5..9), Poisson arrivals at each
offered rate for ``--duration`` seconds, chains of 1..16 products whose
factors are generated on the device; per rate the achieved GFLOP/s and the
p50 / p99 request latency, under continuous batching and, on the same
arrivals, in lock-step rounds (the paper's batched approach); ``value`` is the
continuous-batching GFLOP/s at the highest rate.

``--workload gram15`` times the complex batched GEMM on the paper's
entanglement-entropy product: 10,000 Hermitian Gram products C = Psi Psi^H
with Psi of 2^8 x 2^7 complex entries (S = 15 spins), binary64, counting
8 m n k real flops per instance; ``--workload gram21`` the same for 64
products with Psi of 2^11 x 2^10 (S = 21), checked on sampled rows of C.

``--workload config1`` (1000 x 32^3, beta 0) and ``--workload vb8`` (the
variable-size batch with leading dimensions padded to multiples of 8) are
secondary lines over one part; with ``--cold`` (the default for config1) each
part is also timed with the last-level cache flushed before every launch
(``ms_cold``, ``roofline_frac_cold``), since config1's 24.6 MB of operands
otherwise stay cache-resident between launches.

``--workload gate21`` times the two-spin gate on 64 states of S = 21 spins
(2^21 binary64 complex amplitudes each, 32 MiB), a new seeded site and gate
per state; HBM-bound (each state read and written once per step).

``--workload ksweep`` is a diagnostic of the uniform path: batches of 256^2
and 512^2 C blocks at one fixed flop count, k from 32 to 4096, beta 0 and 1;
at fixed flops the number of tiles falls as k grows, which separates each
tile's fixed cost from the rate of the k loop.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_FP64 = 78.6e12      # MI355X published FP64 (vector and matrix), flop/s
PEAK_HBM = 8.0e12        # MI355X published HBM3E bandwidth, bytes/s
PEAK_FP32_MFMA = 157.3e12  # dense binary32 matrix cores
PEAK_BF16_MFMA = 2.5e15    # dense bfloat16 matrix cores
PEAK_INT8_MFMA = 5.0e15    # dense int8 matrix cores (operations per second)
FP64_ACCURACY = 1e-13      # relative Frobenius error that counts as binary64 accuracy
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


def parse_mode(name: str):
    """'fp64' | 'fp32' | 'bf16' | 'emu<s>' | 'i8emu<s>' | 'f32emu<s>' -> (bg_mode_t value,
    slices)."""
    fixed = {"fp64": (0, 0), "fp32": (1, 0), "bf16": (2, 0)}
    if name in fixed:
        return fixed[name]
    if name.startswith("emu") and name[3:].isdigit() and 1 <= int(name[3:]) <= 8:
        return (3, int(name[3:]))
    if name.startswith("f32emu") and name[6:].isdigit() and 1 <= int(name[6:]) <= 8:
        return (5, int(name[6:]))
    if name.startswith("i8emu") and name[5:].isdigit() and 1 <= int(name[5:]) <= 8:
        return (4, int(name[5:]))
    raise ValueError("unknown precision mode " + name)


def mode_launch(h, p, mode):
    code, slices = mode
    pA, pB, pC = p.pointers()
    st = h.gemm_batched_mode_raw(code, slices, "N", "N", p.m, p.n, p.k, p.alpha, pA.data_ptr(),
                                 p.A.shape[-1], pB.data_ptr(), p.B.shape[-1], p.beta,
                                 pC.data_ptr(), p.C.shape[-1], p.batch)
    if st != 0:
        raise RuntimeError("mode launch of %s failed with status %d" % (p.name, st))


def mode_flops(p, mode):
    """(binary64-equivalent flops, flops the matrix cores execute) per launch."""
    f = p.flops
    code, s = mode
    return f, (f * s * (s + 1) / 2 if code in (3, 4, 5) else f)


def mode_peak(mode):
    return {0: PEAK_FP64, 1: PEAK_FP32_MFMA, 2: PEAK_BF16_MFMA, 3: PEAK_BF16_MFMA,
            4: PEAK_INT8_MFMA, 5: PEAK_FP32_MFMA}[mode[0]]


def precision_bench(args, h, parts):
    """The config4 line: every mode in --modes on the wide-exponent batch."""
    import numpy as np
    import torch
    import oracle
    from oracle import precision as P
    from paper_2203_09353_amd import inputs
    from paper_2203_09353_amd.workloads import host_instance

    p = parts[0]
    names = args.modes.split(",")
    if "fp64" not in names:
        names = ["fp64"] + names          # the baseline every gain is measured against
    modes = [parse_mode(n) for n in names]
    # accuracy is judged on at least 32 sampled instances
    idx = inputs.permutation(11, 4, p.batch)[:max(32, args.check)].tolist()
    picks = []
    for i in idx:
        A, B, _ = host_instance(p, i)
        Am, Bm = np.ascontiguousarray(A[:, :p.m].T), np.ascontiguousarray(B[:, :p.k].T)
        C = np.zeros((p.n, p.m))
        oracle.gemm("N", "N", p.m, p.n, p.k, 1.0, A, A.shape[-1], B, B.shape[-1], 0.0, C, p.m)
        picks.append((i, Am, Bm, C.T.copy(), P.dot2_gemm(Am, Bm), np.abs(Am) @ np.abs(Bm)))
    log("references for %d sampled instances ready" % len(picks))
    oracle_floor = max(P.relative_errors(f64, d2)[0] for _, _, _, f64, d2, _ in picks)
    stream = torch.cuda.current_stream()
    rows = []
    for name, mode in zip(names, modes):
        p.C.fill_(float("nan"))
        mode_launch(h, p, mode)
        torch.cuda.synchronize()
        fro, fro64, comp, exact = [], [], [], None
        for j, (i, Am, Bm, f64, d2, mag) in enumerate(picks):
            G = np.ascontiguousarray(p.C[i].cpu().numpy()[:, :p.m].T)
            fro.append(P.relative_errors(G, d2)[0])
            fro64.append(P.relative_errors(G, f64)[0])
            comp.append(float(np.max(np.abs(G - d2) / np.where(mag > 0, mag, 1.0))))
            if mode[0] in (3, 4, 5) and j == 0:
                emu = P.int8_emulated_gemm if mode[0] == 4 else P.emulated_gemm
                ref = emu(Am, Bm, mode[1])
                exact = bool(np.array_equal(G.view(np.int64), ref.view(np.int64)))
        for _ in range(args.warmup):
            mode_launch(h, p, mode)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            mode_launch(h, p, mode)
            e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / args.steps
        ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
        f64_flops, core_flops = mode_flops(p, mode)
        row = {"mode": name, "ms": round(ms, 4), "wall_ms": round(wall * 1e3, 4),
               "gflops_fp64_equiv": round(f64_flops / (ms * 1e-3) / 1e9, 1),
               "core_tflops": round(core_flops / (ms * 1e-3) / 1e12, 2),
               "core_peak_frac": round(core_flops / (ms * 1e-3) / mode_peak(mode), 4),
               "max_rel_fro_vs_dot2": float("%.3e" % max(fro)),
               "mean_rel_fro_vs_dot2": float("%.3e" % (sum(fro) / len(fro))),
               "max_rel_fro_vs_fp64_oracle": float("%.3e" % max(fro64)),
               "max_componentwise_vs_dot2": float("%.3e" % max(comp)),
               "fp64_accuracy": bool(max(fro) <= FP64_ACCURACY)}
        if exact is not None:
            row["bit_exact_vs_oracle"] = exact
        log(json.dumps(row))
        rows.append(row)
    ok = [r for r in rows if r["fp64_accuracy"]]
    if not ok:
        # no mode, not even the binary64 path, met the rule: there is no
        # figure "at FP64 accuracy" to report
        log("no precision mode reached binary64 accuracy")
        sys.exit(3)
    best = max(ok, key=lambda r: r["gflops_fp64_equiv"])
    bmode = parse_mode(best["mode"])
    sec = best["ms"] * 1e-3
    core = mode_flops(p, bmode)[1]
    roof = {"bound": "mfma", "achieved": round(core / sec / 1e12, 3),
            "peak": mode_peak(bmode) / 1e12, "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = None
    roof["kernel"] = "%s (%s)" % (p.name, best["mode"])
    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle of mode %s on a sample" % best["mode"])
        cpu = precision_cpu_baseline(p, bmode, args.cpu_seconds)
    dtype = {0: "f64", 1: "f32", 2: "bf16", 3: "bf16 slices (f32 sums, f64 recombination)",
             4: "int8 slices (int32 sums, f64 recombination)",
             5: "8-bit digit slices on f32 matrix cores (f32 sums, f64 recombination)"}[bmode[0]]
    out = {"metric": METRIC, "value": best["gflops_fp64_equiv"], "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded counter-based s m 2^e, m in [1,2), e in -20..20)",
           "config": {"workload": "config4", "parts": "%s x%d" % (p.name, p.batch),
                      "mode": best["mode"],
                      "accuracy_rule": "max rel Frobenius vs Dot2 <= %g" % FP64_ACCURACY},
           "roofline": roof, "cpu_baseline": cpu, "modes": rows,
           "gain_vs_fp64": next((round(best["gflops_fp64_equiv"] / r["gflops_fp64_equiv"], 3)
                                 for r in rows if r["mode"] == "fp64"), None),
           "fp64_oracle_floor_vs_dot2": float("%.3e" % oracle_floor)}
    print(json.dumps(out), flush=True)


def precision_cpu_baseline(p, mode, seconds):
    """The oracle of `mode` (binary64 C oracle or the precision oracle) on the
    first instances of the part, for about `seconds` of work."""
    import numpy as np
    import oracle
    from oracle import precision as P
    from paper_2203_09353_amd.workloads import host_instance

    threads = len(os.sched_getaffinity(0))
    t, n = 0.0, 0
    used = 1
    while t < seconds and n < p.batch:
        A, B, _ = host_instance(p, n)
        if mode[0] == 0:
            C = np.zeros((p.n, p.m))
            t0 = time.perf_counter()
            oracle.gemm("N", "N", p.m, p.n, p.k, 1.0, A, A.shape[-1], B, B.shape[-1], 0.0, C, p.m)
            t += time.perf_counter() - t0
        else:
            Am, Bm = np.ascontiguousarray(A[:, :p.m].T), np.ascontiguousarray(B[:, :p.k].T)
            t0 = time.perf_counter()
            if mode[0] in (3, 5):
                P.emulated_gemm(Am, Bm, mode[1])
            elif mode[0] == 4:
                P.int8_emulated_gemm(Am, Bm, mode[1])
            else:
                P.reference_product(Am, Bm, "fp32" if mode[0] == 1 else "bf16")
                used = threads
            t += time.perf_counter() - t0
        n += 1
    flops = 2.0 * p.m * p.n * p.k * n
    return {"value": round(flops / t / 1e9, 3), "unit": "GFLOP/s", "cores": used,
            "kind": "oracle",
            "sample": "first %d of %d instances of %s, one at a time, %.1f s" % (
                n, p.batch, p.name, t)}


def serving_bench(args, h):
    """The config5 line: the request loop at each offered rate."""
    import numpy as np
    import torch
    from oracle import serving
    from paper_2203_09353_amd import serve

    clients, seed = 64, 5
    sizes = serve.client_sizes(seed, clients)
    srv = serve.Server(h, sizes, seed=seed, budget=64 << 30)
    rows = []
    try:
        # warm-up: one short schedule
        a, c, l = serve.requests(seed + 100, clients, 2000.0, 0.05)
        srv.run(a, c, l)
        lockstep_rows, vtick_rows = [], []
        for rate in [float(x) for x in args.rates.split(",")]:
            a, c, l = serve.requests(seed, clients, rate, args.duration)
            # the same arrivals under continuous batching (the paper's tasked
            # approach), in lock-step rounds (its batched approach), and under
            # continuous batching with each tick issued as one variable-size
            # launch instead of one uniform launch per client size
            for policy, tick, out_rows in (
                    (serve.POLICY_CONTINUOUS, serve.TICK_PER_SIZE, rows),
                    (serve.POLICY_LOCKSTEP, serve.TICK_PER_SIZE, lockstep_rows),
                    (serve.POLICY_CONTINUOUS, serve.TICK_VBATCHED, vtick_rows)):
                srv.reset()
                srv.set_policy(policy)
                srv.set_tick_launch(tick)
                st, fi, ticks = srv.run(a, c, l)
                pool, peak, waits = srv.memory_stats()
                n = sizes[c].astype(np.float64)
                flops = float((2.0 * n ** 3 * l).sum())
                wall = float(fi.max())
                lat = (fi - a) * 1e3
                row = {"offered_req_s": rate, "requests": int(len(a)),
                       "achieved_req_s": round(len(a) / wall, 1),
                       "gflops": round(flops / wall / 1e9, 1),
                       "p50_ms": round(float(np.percentile(lat, 50)), 3),
                       "p99_ms": round(float(np.percentile(lat, 99)), 3),
                       "mean_ms": round(float(lat.mean()), 3),
                       "ticks": int(ticks), "mean_batch": round(float(l.sum()) / max(ticks, 1), 2),
                       "wall_s": round(wall, 3), "factor_pool_peak_bytes": int(peak),
                       "memory_waits": int(waits)}
                log(("lock step " if policy == serve.POLICY_LOCKSTEP else
                     "continuous, one variable-size launch per tick " if tick == serve.TICK_VBATCHED
                     else "continuous ") + json.dumps(row))
                out_rows.append(row)
            srv.set_policy(serve.POLICY_CONTINUOUS)
            srv.set_tick_launch(serve.TICK_PER_SIZE)
        # baseline: the same loop serving one request at a time (no batching
        # across clients), on a 0.1 s slice of the highest offered rate
        srv.reset()
        srv.set_max_active(1)
        a1, c1, l1 = serve.requests(seed, clients, float(args.rates.split(",")[-1]), 0.1)
        st1, fi1, _ = srv.run(a1, c1, l1)
        srv.set_max_active(0)
        n1 = sizes[c1].astype(np.float64)
        wall1 = float(fi1.max())
        lat1 = (fi1 - a1) * 1e3
        serial = {"offered_req_s": float(args.rates.split(",")[-1]), "requests": int(len(a1)),
                  "achieved_req_s": round(len(a1) / wall1, 1),
                  "gflops": round(float((2.0 * n1 ** 3 * l1).sum()) / wall1 / 1e9, 1),
                  "p50_ms": round(float(np.percentile(lat1, 50)), 3),
                  "p99_ms": round(float(np.percentile(lat1, 99)), 3), "wall_s": round(wall1, 3)}
        log("one request at a time: " + json.dumps(serial))
        srv.reset()
        a, c, l = serve.requests(seed, clients, float(args.rates.split(",")[-1]), args.duration)
        srv.run(a, c, l)
        # lock-step annealing sweeps (every client 16 products per sweep, 100
        # sweeps), launches issued one by one vs replayed from a HIP graph
        sw = {}
        for mode in ("eager", "graph"):
            srv.reset()
            secs = srv.sweeps(100, 16, graph=(mode == "graph"))
            fl = float((2.0 * sizes.astype(np.float64) ** 3).sum()) * 16 * 100
            sw[mode] = {"seconds": round(secs, 4), "gflops": round(fl / secs / 1e9, 1)}
        sw["graph_speedup"] = round(sw["eager"]["seconds"] / sw["graph"]["seconds"], 3)
        log("sweeps: " + json.dumps(sw))
        # the same sweeps for 64 clients of 32 x 32 states, where each launch
        # is short and the launch cost shows
        small = serve.Server(h, [32] * clients, seed=seed + 1)
        try:
            sws = {}
            for mode in ("eager", "graph"):
                small.sweeps(2, 16, graph=(mode == "graph"))     # warm-up
                small.reset()
                secs = small.sweeps(100, 16, graph=(mode == "graph"))
                fl = 2.0 * 32 ** 3 * clients * 16 * 100
                sws[mode] = {"seconds": round(secs, 5), "gflops": round(fl / secs / 1e9, 1)}
            sws["graph_speedup"] = round(sws["eager"]["seconds"] / sws["graph"]["seconds"], 3)
            log("sweeps, 32 x 32 states: " + json.dumps(sws))
        finally:
            small.close()
        srv.reset()
        srv.run(a, c, l)
        # parity: one client of the last run against the CPU replay
        prods = serving.products_per_client(clients, c, l)
        cl = int(np.argmin(np.where(prods > 0, sizes * 1000 + prods, 1 << 40)))
        S, p = srv.state(cl)
        ref = serving.final_state(seed, cl, int(sizes[cl]), int(p))
        parity = float(np.linalg.norm(S - ref) / np.linalg.norm(ref))
    finally:
        srv.close()
    top = rows[-1]
    roof = {"bound": "mfma", "achieved": round(top["gflops"] / 1e3, 3), "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof["traffic"] = None
    roof["kernel"] = "request loop at %g req/s (factor generation + batched GEMMs)" % top[
        "offered_req_s"]
    cpu = None
    if not args.no_cpu:
        log("timing the CPU replay on a sample")
        t0 = time.perf_counter()
        done, fl = 0, 0.0
        order = np.argsort(sizes[c], kind="stable")
        for r in order:
            nn = int(sizes[c[r]])
            serving.final_state(seed, int(c[r]), nn, int(l[r]))
            done += 1
            fl += 2.0 * nn ** 3 * l[r]
            if time.perf_counter() - t0 > args.cpu_seconds:
                break
        t = time.perf_counter() - t0
        cpu = {"value": round(fl / t / 1e9, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
               "sample": "%d requests of the last rate, smallest states first, factors from the "
                         "Philox oracle, %.1f s" % (done, t)}
    out = {"metric": METRIC, "value": top["gflops"], "unit": "GFLOP/s", "n_gpus": 1,
           "steps": len(rows), "warmup": 1, "ms_per_step": round(top["wall_s"] * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (Poisson arrivals, factors from a Philox4x64-10 stream on the device)",
           "config": {"workload": "config5", "clients": clients,
                      "state_sizes": sorted(set(int(x) for x in sizes)),
                      "duration_s": args.duration},
           "roofline": roof, "cpu_baseline": cpu, "rates": rows,
           "lockstep_rates": lockstep_rows, "vbatched_tick_rates": vtick_rows,
           "continuous_vs_lockstep": {
               "throughput_at_top_rate": round(top["achieved_req_s"] /
                                               lockstep_rows[-1]["achieved_req_s"], 3),
               "mean_latency_ratio_per_rate": [round(r["mean_ms"] / q["mean_ms"], 3)
                                               for r, q in zip(rows, lockstep_rows)]},
           "hbm_budget_bytes": 64 << 30, "one_at_a_time": serial,
           "sweeps_100x16": sw, "sweeps_100x16_32x32_states": sws,
           "batching_gain": round(top["achieved_req_s"] / serial["achieved_req_s"], 2),
           "parity_rel_fro_one_client": parity}
    print(json.dumps(out), flush=True)


GRAM = {15: 10_000, 21: 64}     # spins S -> instances of the Gram product


def gram_bench(args, h, S=15):
    """The gram<S> line: C_i = Psi_i Psi_i^H, Psi_i of 2^ceil(S/2) x
    2^floor(S/2) complex (256 x 128 at S = 15, 2048 x 1024 at S = 21)."""
    import numpy as np
    import torch
    import oracle
    from paper_2203_09353_amd import inputs, bgemm as bg

    batch, rows, cols = GRAM[S], 2 ** ((S + 1) // 2), 2 ** (S // 2)
    seed = 6
    re = torch.empty(batch, cols, rows, dtype=torch.float64, device="cuda")
    im = torch.empty_like(re)
    for X, st in ((re, 0), (im, 1)):
        flat = X.view(-1)
        for off in range(0, flat.numel(), 1 << 26):
            n = min(1 << 26, flat.numel() - off)
            flat[off:off + n] = inputs.uniform_flat(seed, st, off, n, device="cuda")
    Psi = torch.complex(re, im)
    del re, im
    C = torch.zeros(batch, rows, rows, dtype=torch.complex128, device="cuda")
    perm = inputs.permutation(seed, 9, batch).cuda()
    pP = bg.pointer_array(Psi)[perm]
    pC = bg.pointer_array(C)[perm]

    def launch():
        st = h.zgemm_batched_raw("N", "C", rows, rows, cols, 1.0, pP.data_ptr(), rows,
                                 pP.data_ptr(), rows, 0.0, pC.data_ptr(), rows, batch)
        if st != 0:
            raise RuntimeError("bg_zgemm_batched failed with status %d" % st)

    launch()
    torch.cuda.synchronize()
    worst = 0.0
    nsel = min(rows, 16)      # sampled rows of C: the oracle on those rows of Psi
    for i in inputs.permutation(11, 6, batch)[:max(1, args.check)].tolist():
        P = Psi[i].cpu().numpy()                                     # (cols, rows) storage
        sel = np.sort(inputs.permutation(13, i, rows)[:nsel].numpy())
        Psel = np.ascontiguousarray(P[:, sel])                       # nsel x cols, column-major
        ref = np.zeros((1, rows, nsel), dtype=np.complex128)         # nsel x rows result
        oracle.zgemm_batched("N", "C", nsel, rows, cols, 1.0, Psel[None], P[None], 0.0, ref)
        got = C[i].cpu().numpy()[:, sel]                             # rows sel of C
        worst = max(worst, float(np.linalg.norm(got - ref[0]) / np.linalg.norm(ref[0])))
    log("sampled parity (max rel Frobenius): %.3e" % worst)
    for _ in range(args.warmup):
        launch()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        launch()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    flops = 8.0 * rows * rows * cols * batch
    tf = flops / (ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(tf, 3), "peak": PEAK_FP64 / 1e12,
            "unit": "TFLOP/s", "frac": round(tf * 1e12 / PEAK_FP64, 4), "traffic": None,
            "kernel": "k_zgemm (N, C) %d x %d x %d complex" % (rows, rows, cols)}
    cpu = None
    if not args.no_cpu:
        log("timing the complex oracle on a sample")
        threads = len(os.sched_getaffinity(0))
        if rows <= 256:
            n = 1
            while True:
                P = Psi[:n].cpu().numpy()
                ref = np.zeros((n, rows, rows), dtype=np.complex128)
                t1 = time.perf_counter()
                oracle.zgemm_batched("N", "C", rows, rows, cols, 1.0, P, P, 0.0, ref,
                                     nthreads=threads)
                t = time.perf_counter() - t1
                if t > args.cpu_seconds / 4 or n >= batch:
                    break
                n = min(batch, n * 4)
            cpu = {"value": round(8.0 * rows * rows * cols * n / t / 1e9, 3), "unit": "GFLOP/s",
                   "cores": min(threads, n), "kind": "oracle",
                   "sample": "first %d of %d instances, %.1f s" % (n, batch, t)}
        else:
            # one instance is too long for the time box: the first r rows of
            # C of the first instance, r doubling until the time box is used
            P = Psi[0].cpu().numpy()
            r = 16
            while True:
                Psel = np.ascontiguousarray(P[:, :r])
                ref = np.zeros((1, rows, r), dtype=np.complex128)
                t1 = time.perf_counter()
                oracle.zgemm_batched("N", "C", r, rows, cols, 1.0, Psel[None], P[None], 0.0, ref,
                                     nthreads=threads)
                t = time.perf_counter() - t1
                if t > args.cpu_seconds / 4 or r >= rows:
                    break
                r = min(rows, r * 2)
            # the oracle parallelises over instances: one instance, one thread
            cpu = {"value": round(8.0 * r * rows * cols / t / 1e9, 3), "unit": "GFLOP/s",
                   "cores": 1, "kind": "oracle",
                   "sample": "first %d of %d rows of C of one instance, %.1f s" % (r, rows, t)}
    out = {"metric": METRIC, "value": round(flops / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "wall_ms_per_step": round(wall * 1e3, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c128 (f64 pairs)",
           "data": "synthetic (seeded counter-based uniform[-1,1) real and imaginary parts)",
           "config": {"workload": "gram%d" % S, "instances": batch, "psi": [rows, cols],
                      "op": "C = Psi Psi^H"},
           "roofline": roof, "cpu_baseline": cpu, "parity_max_rel_fro": worst}
    print(json.dumps(out), flush=True)


def gate_bench(args, h):
    """The gate21 line: in-place two-spin gates on 64 states of 2^21 amplitudes."""
    import numpy as np
    import torch
    from oracle import gates as G
    from paper_2203_09353_amd import inputs

    S, batch = 21, 64
    amps = 1 << S
    psi = torch.empty(batch, amps, dtype=torch.complex128, device="cuda")
    view = torch.view_as_real(psi).view(-1)
    for off in range(0, view.numel(), 1 << 26):
        n = min(1 << 26, view.numel() - off)
        view[off:off + n] = inputs.uniform_flat(7, 0, off, n, device="cuda")
    g = inputs.gaussian_flat(7, 2, 0, batch * 32).view(batch, 32).numpy()
    U = np.stack([G.haar_unitary(g[i, :16], g[i, 16:]) for i in range(batch)])
    Ud = torch.tensor(U).cuda()
    u = (inputs.uniform_flat(7, 3, 0, batch).numpy() + 1.0) * 0.5
    sites = torch.tensor(np.minimum((u * (S - 1)).astype(np.int32), S - 2)).cuda()
    # parity: one state, one step, against the oracle
    before = psi[5].cpu().numpy()
    h.zgate2(S, sites, Ud, psi)
    torch.cuda.synchronize()
    ref = G.apply_gate(before, S, int(sites[5]), U[5])
    parity = float(np.abs(psi[5].cpu().numpy() - ref).max())
    for _ in range(args.warmup):
        h.zgate2(S, sites, Ud, psi)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        h.zgate2(S, sites, Ud, psi)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    nbytes = 2.0 * 16 * amps * batch            # every amplitude read and written once
    gbps = nbytes / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": round(gbps * 1e9 / PEAK_HBM, 4), "traffic": None,
            "kernel": "k_gate2 (64 states of 2^21 amplitudes)"}
    cpu = None
    if not args.no_cpu:
        st = psi[0].cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 10.0):
            st = G.apply_gate(st, S, int(sites[0]), U[0])
            reps += 1
        t = time.perf_counter() - t0
        cpu = {"value": round(2.0 * 16 * amps * reps / t / 1e9, 3), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "sample": "%d gates on one 2^21-amplitude state, %.1f s" % (reps, t)}
    out = {"metric": "two-spin gate GB/s on 2^21-amplitude states, % HBM roofline",
           "value": round(gbps, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c128 (f64 pairs)",
           "data": "synthetic (seeded uniform amplitudes, Haar 4x4 unitaries, seeded sites)",
           "config": {"workload": "gate21", "states": batch, "spins": S},
           "roofline": roof, "cpu_baseline": cpu, "parity_max_abs": parity}
    print(json.dumps(out), flush=True)


def ksweep_bench(args, h):
    """The ksweep line: uniform 'N','N' batches of 256^2 and 512^2 C blocks
    at a fixed 6.7e11 flop (20,000 x 256^3 x 2), k from 32 to 4096, with
    beta 0 and 1.  At fixed flops the tile count falls as k grows, so the
    rate against k separates the per-tile cost (pipeline fill, epilogue,
    the C read with beta != 0) from the k-loop's own rate."""
    import torch
    from paper_2203_09353_amd import workloads
    rows = []
    worst = 0.0
    for (m, n) in ((256, 256), (512, 512)):
        for k in (32, 64, 128, 256, 512, 1024, 2048, 4096):
            batch = max(1, int(20000 * 256 ** 3 / (m * n * k)))
            row = {"m": m, "n": n, "k": k, "batch": batch}
            for beta in (0.0, 1.0):
                p = workloads.uniform_part("k%d" % k, batch, m, n, k, 1.0, beta, 12)
                if args.check > 0:
                    worst = max(worst, sampled_parity(h, [p], 1)[p.name])
                for _ in range(max(1, args.warmup)):
                    part_launch(h, p)
                stream = torch.cuda.current_stream()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.steps)]
                torch.cuda.synchronize()
                for e0, e1 in ev:
                    e0.record(stream)
                    part_launch(h, p)
                    e1.record(stream)
                torch.cuda.synchronize()
                ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
                key = "beta%d" % int(beta)
                row[key + "_ms"] = round(ms, 4)
                row[key + "_tflops"] = round(p.flops / (ms * 1e-3) / 1e12, 2)
                del p
                torch.cuda.empty_cache()
            rows.append(row)
            log(json.dumps(row))
    best = max(max(r["beta0_tflops"], r["beta1_tflops"]) for r in rows)
    out = {"metric": "uniform FP64 batched GEMM TFLOP/s against k at fixed flops",
           "value": best, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded uniform[-1,1))",
           "config": {"workload": "ksweep", "flops_per_batch": 2 * 20000 * 256 ** 3},
           "rows": rows, "parity_max_rel_fro": worst}
    print(json.dumps(out), flush=True)


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


def cold_part_ms(h, parts, reps, flush_bytes=1 << 30):
    """Per-part event-timed milliseconds with the caches cold: before each
    repetition a 1 GiB buffer (four times the 256 MB last-level cache) is
    overwritten, then each part is launched once."""
    import torch
    flush = torch.empty(flush_bytes // 8, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in parts] for _ in range(reps)]
    for r in range(reps):
        for j, p in enumerate(parts):
            flush.fill_(float(r + j))
            ev[r][j][0].record(stream)
            part_launch(h, p)
            ev[r][j][1].record(stream)
    torch.cuda.synchronize()
    del flush
    return [sum(ev[r][j][0].elapsed_time(ev[r][j][1]) for r in range(reps)) / reps
            for j in range(len(parts))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="config2+vb")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--check", type=int, default=3,
                    help="sampled parity instances per part (config4: at least 32)")
    ap.add_argument("--cold", action="store_true",
                    help="also time every part with cold caches (default for config1)")
    ap.add_argument("--modes", default="fp64,fp32,bf16,emu3,emu6,emu7,f32emu3,f32emu6,i8emu6,i8emu7,"
                                        "i8emu8",
                    help="precision modes timed by --workload config4")
    ap.add_argument("--rates", default="1000,5000,20000,50000",
                    help="offered request rates (per second) for --workload config5")
    ap.add_argument("--duration", type=float, default=2.0,
                    help="seconds of arrivals per rate for --workload config5")
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
    if args.workload == "config5":
        serving_bench(args, h)
        return
    if args.workload in ("gram15", "gram21"):
        gram_bench(args, h, int(args.workload[4:]))
        return
    if args.workload == "gate21":
        gate_bench(args, h)
        return
    if args.workload == "ksweep":
        ksweep_bench(args, h)
        return
    log("building workload %s" % args.workload)
    t0 = time.perf_counter()
    parts = workloads.build(args.workload, "cuda")
    torch.cuda.synchronize()
    log("built in %.1f s; device memory %.1f GB" % (time.perf_counter() - t0,
                                                     torch.cuda.memory_allocated() / 1e9))

    if args.workload == "config4":
        precision_bench(args, h, parts)
        return

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
    if args.cold or args.workload in ("config1", "u32"):
        log("timing with cold caches")
        for row, p, ms in zip(part_rows, parts, cold_part_ms(h, parts, max(3, args.steps))):
            row["ms_cold"] = round(ms, 4)
            if hasattr(p, "per_instance_roofline_s"):
                t_roof = p.per_instance_roofline_s(PEAK_FP64, PEAK_HBM)
            else:
                t_roof = max(p.flops / PEAK_FP64, p.bytes / PEAK_HBM)
            row["roofline_frac_cold"] = round(t_roof / (ms * 1e-3), 4)
            row["gbps_cold"] = round(p.bytes / (ms * 1e-3) / 1e9, 1)
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
