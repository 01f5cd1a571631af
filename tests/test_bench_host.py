"""Host-side logic of bench.py and the profile summaries (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2203_09353_amd import profile_summary

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_reported_only_for_current_kernels(tmp_path, monkeypatch):
    blob = {"kernel_source_sha256": profile_summary.kernel_source_hash(), "workload": "config2+vb",
            "parts": {"s512": {"read_bytes": 3.0e10, "write_bytes": 1.0e10}}}
    p = tmp_path / "summary.md"
    p.write_text("# x\n\n```json\n" + json.dumps(blob) + "\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(p))
    t = bench.measured_traffic("s512", "config2+vb")
    assert t["bytes"] == 4.0e10 and t["read"] == 3.0e10
    assert bench.measured_traffic("s512", "vb") is None          # other workload
    assert bench.measured_traffic("u64", "config2+vb") is None   # part not measured
    blob["kernel_source_sha256"] = "0" * 64                      # kernels changed since
    p.write_text("```json\n" + json.dumps(blob) + "\n```\n")
    assert bench.measured_traffic("s512", "config2+vb") is None


def test_committed_summary_parses():
    t = profile_summary.load_traffic(bench.TRAFFIC_SUMMARY)
    assert t is not None and t["workload"] == "config2+vb"
    for part in ("u64", "u256", "s512", "vb"):
        assert t["parts"][part]["read_bytes"] > 0


def test_part_attribution_of_dispatches():
    assert profile_summary.part_of("void bg::k_vb_exec<bg::Cfg<128, 64, 16>>", 0) == "vb"
    assert profile_summary.part_of("void bg::k_uniform<bg::Cfg<64, 64, 16>>", 0) == "u64"
    assert profile_summary.part_of("void bg::k_uniform<bg::Cfg<128, 64, 16>>", 0) == "u256"
    assert profile_summary.part_of("void bg::k_uniform<bg::Cfg<128, 64, 16>>", 1) == "s512"


def test_padded_variable_size_workload_across_fill_groups():
    """ld rounded up to 8: every instance's payload (also past the first fill
    group) is the generator's, padding rows are NaN."""
    from paper_2203_09353_amd import inputs, workloads
    p = workloads.vb_part("vb8", 300, 1.0, 0.5, 4, pad8=True, device="cpu", group=128)
    ms, ns, ks, la, lb, lc = p.sizes_host
    pay = ms * ks
    for i in (0, 127, 128, 200, p.batch - 1):
        A, _, _ = workloads.host_instance(p, i)
        m, k = int(ms[i]), int(ks[i])
        assert int(la[i]) % 8 == 0 and int(la[i]) >= m
        ref = inputs.uniform_flat(4, 0, int(pay[:i].sum()), m * k).view(k, m).numpy()
        assert np.array_equal(A[:, :m], ref)
        assert np.isnan(A[:, m:]).all()
