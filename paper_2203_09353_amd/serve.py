"""Python binding of the request loop (include/bgserve.h) and the request
workload of the serving benchmark.

Argument marshalling only: the scheduler and the tick loop run in C++ inside
libbgemm.so, the factors are generated and multiplied by its kernels.

Workload (seeded, synthetic; the paper's procedures apply random local gates
and GEMMs to their states, Section III): ``clients`` clients, client c of size
2^k_c with k_c uniform in 5..9; requests arrive as a Poisson process of rate
``rate`` per second over ``duration`` seconds, each for a uniformly chosen
client, with a chain length uniform in 1..16.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import bgemm, inputs

_set = False


def _lib():
    global _set
    L = bgemm.lib()
    if not _set:
        vp, i, d, u64, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_ulonglong, ctypes.c_longlong
        L.bs_create.restype = i
        L.bs_create.argtypes = [vp, i, vp, u64, u64, ctypes.POINTER(vp)]
        L.bs_destroy.restype = i
        L.bs_destroy.argtypes = [vp]
        L.bs_bytes_needed.restype = u64
        L.bs_bytes_needed.argtypes = [i, vp]
        L.bs_reset.restype = i
        L.bs_reset.argtypes = [vp]
        L.bs_run_schedule.restype = i
        L.bs_run_schedule.argtypes = [vp, i, vp, vp, vp, vp, vp, ctypes.POINTER(ll)]
        L.bs_state.restype = i
        L.bs_state.argtypes = [vp, i, vp, ctypes.POINTER(ll)]
        L.bs_fill_factor.restype = i
        L.bs_fill_factor.argtypes = [u64, i, ll, i, vp, vp]
        L.bs_simulate.restype = i
        L.bs_simulate.argtypes = [i, vp, u64, i, i, vp, vp, vp, d, i, vp, vp,
                                  ctypes.POINTER(ll), ctypes.POINTER(ll)]
        L.bs_set_policy.restype = i
        L.bs_set_policy.argtypes = [vp, i]
        L.bs_memory_stats.restype = i
        L.bs_memory_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                      ctypes.POINTER(ll)]
        L.bs_run_sweeps.restype = i
        L.bs_run_sweeps.argtypes = [vp, i, i, i, ctypes.POINTER(d)]
        L.bs_set_max_active.restype = i
        L.bs_set_max_active.argtypes = [vp, i]
        L.bs_set_tick_launch.restype = i
        L.bs_set_tick_launch.argtypes = [vp, i]
        _set = True
    return L


def _arr(x, dtype):
    return np.ascontiguousarray(np.asarray(x, dtype=dtype))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def bytes_needed(sizes) -> int:
    s = _arr(sizes, np.int32)
    return int(_lib().bs_bytes_needed(len(s), _ptr(s)))


POLICY_CONTINUOUS, POLICY_LOCKSTEP = 0, 1
TICK_PER_SIZE, TICK_VBATCHED = 0, 1


def simulate(num_clients, arrivals, clients, lengths, tick_s, max_active=0,
             policy=POLICY_CONTINUOUS, sizes=None, pool_bytes=0, with_waits=False):
    """Host-only replay of the scheduler on a virtual clock (no device):
    returns (start, finish, ticks), plus the memory waits if `with_waits`."""
    a, c, l = _arr(arrivals, np.float64), _arr(clients, np.int32), _arr(lengths, np.int32)
    n = len(a)
    st, fi = np.zeros(n), np.zeros(n)
    ticks, waits = ctypes.c_longlong(), ctypes.c_longlong()
    sz = None if sizes is None else _arr(sizes, np.int32)
    r = _lib().bs_simulate(num_clients, None if sz is None else _ptr(sz), int(pool_bytes),
                           int(policy), n, _ptr(a), _ptr(c), _ptr(l), float(tick_s),
                           int(max_active), _ptr(st), _ptr(fi), ctypes.byref(ticks),
                           ctypes.byref(waits))
    if r != 0:
        raise bgemm.BgemmError("bs_simulate", r)
    if with_waits:
        return st, fi, ticks.value, waits.value
    return st, fi, ticks.value


def fill_factor(seed, client, j, n, out: torch.Tensor):
    """Factor j of a client into a CUDA float64 tensor of n * n elements."""
    assert out.is_cuda and out.dtype == torch.float64 and out.numel() == n * n
    r = _lib().bs_fill_factor(seed, client, j, n, out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    if r != 0:
        raise bgemm.BgemmError("bs_fill_factor", r)


class Server:
    """Request loop on a bgemm handle (its device, torch's current stream)."""

    def __init__(self, handle: bgemm.Handle, sizes, seed: int, budget: int = 0):
        self.L = _lib()
        self.handle = handle
        self.sizes = _arr(sizes, np.int32)
        handle._sync_stream()
        out = ctypes.c_void_p()
        r = self.L.bs_create(handle._h, len(self.sizes), _ptr(self.sizes), seed, budget,
                             ctypes.byref(out))
        if r != 0:
            raise bgemm.BgemmError("bs_create", r)
        self._s = out

    def close(self):
        if getattr(self, "_s", None):
            self.L.bs_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweeps(self, sweeps: int, chain: int, graph: bool):
        """Lock-step annealing sweeps; returns the device seconds."""
        self.handle._sync_stream()
        secs = ctypes.c_double()
        r = self.L.bs_run_sweeps(self._s, int(sweeps), int(chain), 1 if graph else 0,
                                 ctypes.byref(secs))
        if r != 0:
            raise bgemm.BgemmError("bs_run_sweeps", r)
        return secs.value

    def set_max_active(self, k: int):
        """0: continuous batching (default); 1: one request at a time."""
        r = self.L.bs_set_max_active(self._s, int(k))
        if r != 0:
            raise bgemm.BgemmError("bs_set_max_active", r)

    def set_tick_launch(self, mode: int):
        """TICK_PER_SIZE (default: one batched launch per client size) or
        TICK_VBATCHED (one variable-size launch per tick)."""
        r = self.L.bs_set_tick_launch(self._s, int(mode))
        if r != 0:
            raise bgemm.BgemmError("bs_set_tick_launch", r)

    def set_policy(self, policy: int):
        """POLICY_CONTINUOUS (default) or POLICY_LOCKSTEP."""
        r = self.L.bs_set_policy(self._s, int(policy))
        if r != 0:
            raise bgemm.BgemmError("bs_set_policy", r)

    def memory_stats(self):
        """(pool bytes, peak bytes in use, ticks that waited for memory)."""
        pb, pk, w = ctypes.c_ulonglong(), ctypes.c_ulonglong(), ctypes.c_longlong()
        r = self.L.bs_memory_stats(self._s, ctypes.byref(pb), ctypes.byref(pk), ctypes.byref(w))
        if r != 0:
            raise bgemm.BgemmError("bs_memory_stats", r)
        return pb.value, pk.value, w.value

    def reset(self):
        self.handle._sync_stream()
        r = self.L.bs_reset(self._s)
        if r != 0:
            raise bgemm.BgemmError("bs_reset", r)

    def run(self, arrivals, clients, lengths):
        """Runs an open-loop schedule; returns (start, finish, ticks), times in
        seconds from the start of the call."""
        a, c, l = _arr(arrivals, np.float64), _arr(clients, np.int32), _arr(lengths, np.int32)
        n = len(a)
        st, fi = np.zeros(n), np.zeros(n)
        ticks = ctypes.c_longlong()
        self.handle._sync_stream()
        r = self.L.bs_run_schedule(self._s, n, _ptr(a), _ptr(c), _ptr(l), _ptr(st), _ptr(fi),
                                   ctypes.byref(ticks))
        if r != 0:
            raise bgemm.BgemmError("bs_run_schedule", r)
        return st, fi, ticks.value

    def state(self, client):
        """(state as an ordinary n x n array, products applied so far)."""
        n = int(self.sizes[client])
        buf = np.empty(n * n)
        prods = ctypes.c_longlong()
        r = self.L.bs_state(self._s, client, _ptr(buf), ctypes.byref(prods))
        if r != 0:
            raise bgemm.BgemmError("bs_state", r)
        return buf.reshape(n, n).T.copy(), prods.value


def client_sizes(seed: int, clients: int, kmin: int = 5, kmax: int = 9):
    u = inputs.uniform_flat(seed, 10, 0, clients).numpy()
    k = np.clip(np.floor((u + 1.0) * 0.5 * (kmax - kmin + 1)), 0, kmax - kmin).astype(int) + kmin
    return (2 ** k).astype(np.int32)


def requests(seed: int, clients: int, rate: float, duration: float, max_len: int = 16):
    """Poisson arrivals (exponential gaps from the seeded generator), a client
    and a chain length per request: (arrivals, clients, lengths)."""
    n = max(1, int(math.ceil(rate * duration * 1.5)) + 16)
    u = (inputs.uniform_flat(seed, 11, 0, n).numpy() + 1.0) * 0.5     # [0, 1)
    gaps = -np.log1p(-u) / rate
    t = np.cumsum(gaps)
    keep = t < duration
    t = t[keep]
    m = len(t)
    uc = (inputs.uniform_flat(seed, 12, 0, m).numpy() + 1.0) * 0.5
    ul = (inputs.uniform_flat(seed, 13, 0, m).numpy() + 1.0) * 0.5
    cl = np.minimum((uc * clients).astype(np.int32), clients - 1)
    ln = np.minimum((ul * max_len).astype(np.int32), max_len - 1) + 1
    return t, cl, ln
