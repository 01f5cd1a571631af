"""Summarise rocprofv3 output for profiles/: per-kernel average durations
(--kernel-trace --stats) and HBM bytes per part (--pmc FETCH_SIZE and
--pmc WRITE_SIZE, one counter per run), each scaled by what the same counter
reads for the copy kernel of known size.

    python -m paper_2203_09353_amd.profile_summary --stats S.csv --fetch F.csv \\
        --write W.csv --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N \\
        --workload config2+vb --command "..." --out profiles/NAME.md

The fenced JSON block at the end of the output is read by bench.py, which
reports the traffic only while ``kernel_source_sha256`` matches the current
kernel source and tile shapes.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """sha256 over the kernel source and the tuned tile shapes."""
    h = hashlib.sha256()
    for name in ("csrc/bgemm_kernels.hip", "tune_cache.json"):
        p = os.path.join(HERE, name)
        if os.path.exists(p):
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def part_of(kernel_name: str, order: int) -> str:
    """Part of the config2+vb step that a GEMM dispatch belongs to; the two
    128-tile uniform launches come in the order u256, s512."""
    if "k_vb_exec" in kernel_name:
        return "vb"
    if "k_uniform" in kernel_name:
        if "Cfg<64, 64" in kernel_name:
            return "u64"
        if "Cfg<32, 32" in kernel_name:
            return "u32"
        return "u256" if order == 0 else "s512"
    return "other"


def durations_by_part(path: str) -> dict:
    """Average device time per launch of each part from a --kernel-trace CSV:
    dispatches in start order; the 128-tile uniform launches alternate u256,
    s512 (the benchmark's part order); a variable-size launch is its planning
    kernels plus one persistent kernel per class."""
    rows = [r for r in _rows(path) if "bg::" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    tot, launches = {}, {}
    big = 0
    for r in rows:
        name = r["Kernel_Name"]
        ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        if "k_vb_" in name:
            p = "vb"
            if "k_vb_count" in name:
                launches["vb"] = launches.get("vb", 0) + 1
        else:
            order = 0
            if "k_uniform" in name and "Cfg<64, 64" not in name and "Cfg<32, 32" not in name:
                order = big % 2
                big += 1
            p = part_of(name, order)
            launches[p] = launches.get(p, 0) + 1
        tot[p] = tot.get(p, 0.0) + ms
    return {p: (launches.get(p, 0), tot[p] / max(1, launches.get(p, 0))) for p in tot}


def counter_by_part(path: str, counter: str) -> dict:
    out = {}
    rows = [r for r in _rows(path) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    big_seen = 0
    for r in rows:
        name = r["Kernel_Name"]
        order = 0
        if "k_uniform" in name and "Cfg<64, 64" not in name and "Cfg<32, 32" not in name:
            order = big_seen
            big_seen += 1
        p = part_of(name, order)
        out[p] = out.get(p, 0.0) + float(r["Counter_Value"])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--trace", help="kernel-trace CSV of the same run (per-part durations)")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    # copy calibration: bytes each way / counter reading (KiB) of one dispatch
    cf = [float(r["Counter_Value"]) for r in _rows(a.copy_fetch) if r["Counter_Name"] == "FETCH_SIZE"]
    cw = [float(r["Counter_Value"]) for r in _rows(a.copy_write) if r["Counter_Name"] == "WRITE_SIZE"]
    fetch_factor = a.copy_bytes / (cf[-1] * 1024.0)
    write_factor = a.copy_bytes / (cw[-1] * 1024.0)
    fetch = {k: v * 1024.0 * fetch_factor for k, v in counter_by_part(a.fetch, "FETCH_SIZE").items()}
    write = {k: v * 1024.0 * write_factor for k, v in counter_by_part(a.write, "WRITE_SIZE").items()}

    stats = [r for r in _rows(a.stats) if "bg::" in r["Name"]]
    lines = ["# rocprofv3 summary: batched FP64 GEMM kernels, workload %s" % a.workload, "",
             "Commands (run from the repository root on one MI355X):", ""]
    lines += ["    " + c for c in a.command]
    lines += ["", "## Kernel durations (--kernel-trace --stats)", "",
              "| kernel | calls | average ms | total ms |", "|---|---:|---:|---:|"]
    for r in stats:
        name = r["Name"].split("(")[0]
        lines.append("| `%s` | %s | %.3f | %.3f |" % (name, r["Calls"], float(r["AverageNs"]) / 1e6,
                                                     float(r["TotalDurationNs"]) / 1e6))
    if a.trace:
        per = durations_by_part(a.trace)
        lines += ["", "Per part (device time of its kernels per launch; the two 128-tile uniform "
                  "launches of a step are u256 then s512):", "",
                  "| part | launches | average ms per launch |", "|---|---:|---:|"]
        for p in ("u32", "u64", "u256", "s512", "vb"):
            if p in per:
                lines.append("| %s | %d | %.3f |" % (p, per[p][0], per[p][1]))
    lines += ["", "## HBM traffic per launch (--pmc FETCH_SIZE, --pmc WRITE_SIZE)", "",
              "Copy-kernel calibration on %d bytes each way: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f "
              "(counter KiB -> bytes)." % (a.copy_bytes, fetch_factor, write_factor), "",
              "| part | read GB | written GB |", "|---|---:|---:|"]
    parts = [p for p in ("u32", "u64", "u256", "s512", "vb") if p in fetch or p in write]
    for p in parts:
        lines.append("| %s | %.3f | %.3f |" % (p, fetch.get(p, 0) / 1e9, write.get(p, 0) / 1e9))
    blob = {"kernel_source_sha256": kernel_source_hash(), "workload": a.workload,
            "fetch_factor": fetch_factor, "write_factor": write_factor,
            "parts": {p: {"read_bytes": fetch.get(p, 0.0), "write_bytes": write.get(p, 0.0)}
                      for p in parts}}
    lines += ["", "```json", json.dumps(blob, indent=1), "```", ""]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("wrote", a.out)


def load_traffic(path: str):
    """The JSON block of a summary written by main(), or None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    i = text.rfind("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    return json.loads(text[i + 7:j])


if __name__ == "__main__":
    main()
