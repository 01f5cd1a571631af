"""Builds the HIP library libbgemm.so (gfx950) in-tree with hipcc.

    python -m paper_2203_09353_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbgemm.so")
MICRO_LIB = os.path.join(HERE, "libbgemm_microbench.so")
ARCH = os.environ.get("BG_OFFLOAD_ARCH", "gfx950")
SOURCES = [os.path.join(CSRC, f) for f in ("bgemm_api.cpp", "bgemm_kernels.hip", "bgemm_lowp.hip",
                                           "bgemm_complex.hip", "bgemm_gate.hip", "bgemm_emu8.hip", "bgemm_noalloc.hip", "serve.cpp",
                                           "serve_kernels.hip")]

# Packed FP32 instructions are kept out of every device build.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH, "-Wall",
          "-Wno-unused-command-line-argument"]


def _hipcc(sources, out, extra=()):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + COMMON + DEVICE_FLAGS + list(extra) + list(sources) + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + out)
    os.replace(tmp, out)
    return out


def build() -> list[str]:
    from .tune import cached_defines
    # tile shapes chosen by the autotuner (tune_cache.json), if any
    outs = [_hipcc(SOURCES, LIB, extra=cached_defines(ARCH))]
    mb = os.path.join(CSRC, "microbench.hip")
    if os.path.exists(mb):
        outs.append(_hipcc([mb], MICRO_LIB))
    return outs


if __name__ == "__main__":
    for p in build():
        print(p)
