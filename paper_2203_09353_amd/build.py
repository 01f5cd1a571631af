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


# The tile kernels' hand-written stage waits count the direct-to-LDS loads a
# wave has in flight; a register spill would add private-memory loads and
# stores to that count, so any spill in them fails the build.
RESOURCE_REMARKS = ["-Rpass-analysis=kernel-resource-usage"]
COUNTED_WAIT_KERNELS = ("k_uniform", "k_vb_exec")


def kernels_with_scratch(remarks: str, names=COUNTED_WAIT_KERNELS) -> list[str]:
    """Kernels among `names` (substring match on the mangled name) whose
    compiler resource remark reports a nonzero private (scratch) size."""
    bad, current = [], None
    for line in remarks.splitlines():
        if "remark: Function Name: " in line:
            current = line.split("Function Name: ", 1)[1].split()[0]
        elif "ScratchSize [bytes/lane]: " in line and current is not None:
            size = int(line.split("ScratchSize [bytes/lane]: ", 1)[1].split()[0])
            if size > 0 and any(n in current for n in names):
                bad.append(current)
    return bad


def _hipcc(sources, out, extra=(), check_scratch=False):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["hipcc"] + COMMON + DEVICE_FLAGS + list(extra) +
           (RESOURCE_REMARKS if check_scratch else []) + list(sources) + ["-o", tmp])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + out)
    if check_scratch:
        bad = kernels_with_scratch(r.stderr)
        if bad:
            os.remove(tmp)
            raise RuntimeError("register spills in kernels with counted load waits: " +
                               ", ".join(bad))
    os.replace(tmp, out)
    return out


def build() -> list[str]:
    from .tune import cached_defines
    # tile shapes chosen by the autotuner (tune_cache.json), if any
    outs = [_hipcc(SOURCES, LIB, extra=cached_defines(ARCH), check_scratch=True)]
    mb = os.path.join(CSRC, "microbench.hip")
    if os.path.exists(mb):
        outs.append(_hipcc([mb], MICRO_LIB))
    return outs


if __name__ == "__main__":
    for p in build():
        print(p)
