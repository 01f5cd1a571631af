"""Binding of libbgemm_microbench.so: attainable FP64 matrix/vector peaks,
HBM stream bandwidth and a single FP64 MFMA on given fragments.

    python -m paper_2203_09353_amd.microbench      # prints a JSON summary
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbgemm_microbench.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbgemm_microbench.so not built")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.mb_mfma_f64_16x16x4.restype = ctypes.c_int
        L.mb_mfma_f64_16x16x4.argtypes = [vp, vp, vp, vp]
        L.mb_mfma_f32_16x16x4.restype = ctypes.c_int
        L.mb_mfma_f32_16x16x4.argtypes = [vp, vp, vp, vp]
        L.mb_mfma_bf16_16x16x32.restype = ctypes.c_int
        L.mb_mfma_bf16_16x16x32.argtypes = [vp, vp, vp, vp]
        L.mb_mfma_i8_16x16x64.restype = ctypes.c_int
        L.mb_mfma_i8_16x16x64.argtypes = [vp, vp, vp, vp]
        L.mb_mfma_f64_4x4x4.restype = ctypes.c_int
        L.mb_mfma_f64_4x4x4.argtypes = [vp, vp, vp, vp]
        L.mb_fp64_peak_ms.restype = ctypes.c_double
        L.mb_fp64_peak_ms.argtypes = [ctypes.c_int] * 4 + [vp]
        L.mb_i8_peak_ms.restype = ctypes.c_double
        L.mb_i8_peak_ms.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
        L.mb_stream_ms.restype = ctypes.c_double
        L.mb_stream_ms.argtypes = [ctypes.c_int, vp, vp, ctypes.c_longlong, ctypes.c_int,
                                   ctypes.c_int, vp]
        _lib = L
    return _lib


def mfma_once(a, b, c):
    """a, b: 64 per-lane values; c: (64, 4) per-lane accumulators.  Returns
    the (64, 4) result of one v_mfma_f64_16x16x4_f64 (CPU float64 tensor)."""
    dev = torch.device("cuda")
    a = torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
    b = torch.as_tensor(b, dtype=torch.float64).to(dev).contiguous()
    c = torch.as_tensor(c, dtype=torch.float64).to(dev).contiguous()
    d = torch.empty(64, 4, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    assert lib().mb_mfma_f64_16x16x4(a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr()) == 0
    return d.cpu()


def mfma4_once(a, b, c):
    """One v_mfma_f64_4x4x4_4b_f64; a, b, c: 64 per-lane values.  Returns the
    64 results."""
    dev = torch.device("cuda")
    t = [torch.as_tensor(x, dtype=torch.float64).to(dev).contiguous() for x in (a, b, c)]
    d = torch.empty(64, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    assert lib().mb_mfma_f64_4x4x4(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(),
                                   d.data_ptr()) == 0
    return d.cpu()


def mfma_f32_once(a, b, c):
    """One v_mfma_f32_16x16x4_f32: a, b (64,) floats, c (64, 4).  Returns (64, 4)."""
    dev = torch.device("cuda")
    t = [torch.as_tensor(x, dtype=torch.float32).to(dev).contiguous() for x in (a, b, c)]
    d = torch.empty(64, 4, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    assert lib().mb_mfma_f32_16x16x4(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(),
                                     d.data_ptr()) == 0
    return d.cpu()


def mfma_bf16_once(a, b, c):
    """One v_mfma_f32_16x16x32_bf16: a, b (64, 8) values (rounded to bfloat16
    here), c (64, 4) floats.  Returns (64, 4) floats."""
    dev = torch.device("cuda")
    ab = [torch.as_tensor(x, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).to(dev)
          .contiguous() for x in (a, b)]
    ct = torch.as_tensor(c, dtype=torch.float32).to(dev).contiguous()
    d = torch.empty(64, 4, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    assert lib().mb_mfma_bf16_16x16x32(ab[0].data_ptr(), ab[1].data_ptr(), ct.data_ptr(),
                                       d.data_ptr()) == 0
    return d.cpu()


def mfma_i8_once(a, b, c):
    """One v_mfma_i32_16x16x64_i8: a, b (64, 16) int8 values, c (64, 4)
    int32.  Returns (64, 4) int32."""
    dev = torch.device("cuda")
    ab = [torch.as_tensor(x, dtype=torch.int8).to(dev).contiguous() for x in (a, b)]
    ct = torch.as_tensor(c, dtype=torch.int32).to(dev).contiguous()
    d = torch.empty(64, 4, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    assert lib().mb_mfma_i8_16x16x64(ab[0].data_ptr(), ab[1].data_ptr(), ct.data_ptr(),
                                     d.data_ptr()) == 0
    return d.cpu()


def fp64_peak_tflops(kind: str, grid: int | None = None, iters: int = 4000, reps: int = 5):
    """kind: 'mfma' (16x16x4, 4 chains), 'mfma8' (8 chains), 'mfma4x4'
    (4x4x4, 8 chains), 'valu' (vector FMA)."""
    code = {"mfma": 0, "valu": 1, "mfma8": 3, "mfma4x4": 4}[kind]
    props = torch.cuda.get_device_properties(0)
    grid = grid or props.multi_processor_count * 8
    sink = torch.zeros(256, dtype=torch.float64, device="cuda")
    ms = lib().mb_fp64_peak_ms(code, grid, iters, reps, sink.data_ptr())
    waves = grid * 4
    if code in (0, 3):
        chains = 4 if code == 0 else 8
        flop = waves * iters * chains * 2048.0
    elif code == 4:
        flop = waves * iters * 8 * 512.0
    else:
        flop = waves * iters * 8 * 64 * 2.0
    return flop * reps / (ms * 1e-3) / 1e12, ms


def int8_peak_tops(grid: int | None = None, iters: int = 2000, reps: int = 5):
    """int8 matrix-core throughput (v_mfma_i32_16x16x64_i8, 8 chains) in
    TOP/s."""
    props = torch.cuda.get_device_properties(0)
    grid = grid or props.multi_processor_count * 8
    sink = torch.zeros(256, dtype=torch.int32, device="cuda")
    ms = lib().mb_i8_peak_ms(grid, iters, reps, sink.data_ptr())
    ops = grid * 4 * iters * 8 * 32768.0 * reps
    return ops / (ms * 1e-3) / 1e12, ms


STREAM_KINDS = {"copy_stride": 0, "read_stride": 1, "copy": 2, "read": 3, "copy_nt": 4,
                "read_nt": 5}


def stream_gbps(kind: str, nbytes: int = 4 << 30, grid: int | None = None, reps: int = 10):
    """HBM stream bandwidth in GB/s (copies count read + write bytes).  kind:
    'copy' / 'read' (one 32 KB chunk per workgroup), '..._nt' (nontemporal),
    '..._stride' (grid-stride loop over CUs x 16 workgroups)."""
    code = STREAM_KINDS[kind]
    props = torch.cuda.get_device_properties(0)
    grid = grid or props.multi_processor_count * 16
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src) if code % 2 == 0 else src
    sink = torch.zeros(256, dtype=torch.float64, device="cuda")
    ms = lib().mb_stream_ms(code, src.data_ptr(), dst.data_ptr(), nbytes, grid, reps,
                            sink.data_ptr())
    if ms <= 0:
        raise RuntimeError("mb_stream_ms failed")
    quad = (256 * 8 if code >= 2 else 4 * grid * 256) * 16
    nbytes = nbytes // quad * quad
    moved = nbytes * (2 if code % 2 == 0 else 1) * reps
    del src, dst
    return moved / (ms * 1e-3) / 1e9, ms


def summary():
    out = {"device": torch.cuda.get_device_name(0),
           "cus": torch.cuda.get_device_properties(0).multi_processor_count}
    for k in ("mfma", "mfma8", "mfma4x4", "valu"):
        out["fp64_%s_tflops" % k] = round(fp64_peak_tflops(k)[0], 2)
    out["int8_mfma_tops"] = round(int8_peak_tops()[0], 1)
    for k in STREAM_KINDS:
        out["hbm_%s_gbps" % k] = round(stream_gbps(k)[0], 1)
    return out


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "copy":
        # one warm-up and one timed launch of the copy kernel over N bytes: the
        # reference dispatch for scaling HBM byte counters
        nbytes = int(sys.argv[2]) if len(sys.argv) > 2 else 1 << 30
        gbps, ms = stream_gbps("copy", nbytes=nbytes, reps=1)
        print(json.dumps({"copy_bytes_each_way": nbytes, "gbps": round(gbps, 1)}))
    else:
        print(json.dumps(summary()))
