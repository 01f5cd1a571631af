"""CPU oracle for batched dense GEMM -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (plain C, built with gcc
``-O2 -ffp-contract=off -fopenmp``), a literal transcription of the batched
GEMM definition of the paper's Eq. 1 (Section II) with the BLAS conventions
for alpha, beta and the argument rules; see the header of ``oracle.c``.

Matrices are numpy float64 arrays in the shape convention of
``paper_2203_09353_amd.inputs``: one column-major matrix with leading
dimension ``ld`` is an array of shape ``(cols, ld)``; a uniform batch is
``(batch, cols, ld)``.  Arrays must be C-contiguous.

Parity status of each function: pinned (real GEMM: tests/test_oracle_pins.py and
tests/test_oracle_mutants.py; complex GEMM: tests/test_oracle_complex.py, and the
batched complex wrapper: tests/test_oracle_zgemm_batched.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_pp = ctypes.POINTER(ctypes.c_void_p)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no HIP, no shared code)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c99", "-Wall", _SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_check_args.restype = ctypes.c_int
        L.oracle_check_args.argtypes = [ctypes.c_char, ctypes.c_char] + [ctypes.c_int] * 6
        L.oracle_dgemm.restype = ctypes.c_int
        L.oracle_dgemm.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_int]
        L.oracle_dgemm_batched.restype = ctypes.c_int
        L.oracle_dgemm_batched.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           _c_dbl_pp, ctypes.c_int, _c_dbl_pp, ctypes.c_int,
                                           ctypes.c_double, _c_dbl_pp, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int]
        L.oracle_dgemm_vbatched.restype = ctypes.c_int
        L.oracle_dgemm_vbatched.argtypes = [ctypes.c_char, ctypes.c_char, _c_int_p, _c_int_p,
                                            _c_int_p, ctypes.c_double, _c_dbl_pp, _c_int_p,
                                            _c_dbl_pp, _c_int_p, ctypes.c_double, _c_dbl_pp,
                                            _c_int_p, ctypes.c_int, _c_int_p, ctypes.c_int]
        _c_dbl_p = ctypes.POINTER(ctypes.c_double)
        L.oracle_zgemm.restype = ctypes.c_int
        L.oracle_zgemm.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _c_dbl_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_int, _c_dbl_p, ctypes.c_void_p,
                                   ctypes.c_int]
        L.oracle_zgemm_batched.restype = ctypes.c_int
        L.oracle_zgemm_batched.argtypes = [ctypes.c_char, ctypes.c_char, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _c_dbl_p, _c_dbl_pp,
                                           ctypes.c_int, _c_dbl_pp, ctypes.c_int, _c_dbl_p,
                                           _c_dbl_pp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        _lib = L
    return _lib


def _ch(t: str) -> bytes:
    return t.encode()[:1] if t else b"\0"


def max_threads() -> int:
    return lib().oracle_max_threads()


def check_args(transa, transb, m, n, k, lda, ldb, ldc) -> int:
    return lib().oracle_check_args(_ch(transa), _ch(transb), m, n, k, lda, ldb, ldc)


def _ptr(a: np.ndarray) -> int:
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data


def gemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    """One instance on flat/any C-contiguous float64 buffers; C is updated in
    place.  Returns 0 or -(argument number)."""
    r = lib().oracle_dgemm(_ch(transa), _ch(transb), m, n, k, float(alpha), _ptr(A), lda,
                           _ptr(B), ldb, float(beta), _ptr(C), ldc)
    if r == -100:
        raise MemoryError("oracle_dgemm: allocation failed")
    return r


def _ptr_array(mats):
    arr = (ctypes.c_void_p * len(mats))()
    for i, a in enumerate(mats):
        arr[i] = _ptr(a)
    return arr


def _split(x):
    if isinstance(x, np.ndarray) and x.ndim == 3:
        return [x[i] for i in range(x.shape[0])]
    return list(x)


def gemm_batched(transa, transb, m, n, k, alpha, A, B, beta, C, nthreads=0):
    """Uniform batch.  A, B, C: (batch, cols, ld) arrays or lists of (cols, ld)
    arrays; ld is read from the arrays.  C is updated in place."""
    As, Bs, Cs = _split(A), _split(B), _split(C)
    batch = len(Cs)
    assert len(As) == batch and len(Bs) == batch
    ta, tb = transa in "TtCc", transb in "TtCc"
    lda = As[0].shape[-1] if batch else max(1, k if ta else m)
    ldb = Bs[0].shape[-1] if batch else max(1, n if tb else k)
    ldc = Cs[0].shape[-1] if batch else max(1, m)
    r = lib().oracle_dgemm_batched(_ch(transa), _ch(transb), m, n, k, float(alpha),
                                   _ptr_array(As), lda, _ptr_array(Bs), ldb, float(beta),
                                   _ptr_array(Cs), ldc, batch, int(nthreads))
    if r != 0:
        raise ValueError("oracle_dgemm_batched: info %d" % r)


def gemm_vbatched(transa, transb, ms, ns, ks, alpha, As, Bs, beta, Cs,
                  ldas=None, ldbs=None, ldcs=None, nthreads=0) -> np.ndarray:
    """Per-instance sizes.  As, Bs, Cs: lists of (cols, ld) arrays; ld arrays
    default to the arrays' second dimension.  Returns the per-instance info
    array (0 = computed, -(argument number) = rejected, C untouched)."""
    batch = len(Cs)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    ldas = np.ascontiguousarray([a.shape[-1] for a in As] if ldas is None else ldas, dtype=np.int32)
    ldbs = np.ascontiguousarray([b.shape[-1] for b in Bs] if ldbs is None else ldbs, dtype=np.int32)
    ldcs = np.ascontiguousarray([c.shape[-1] for c in Cs] if ldcs is None else ldcs, dtype=np.int32)
    info = np.zeros(batch, dtype=np.int32)
    ip = lambda a: a.ctypes.data_as(_c_int_p)
    r = lib().oracle_dgemm_vbatched(_ch(transa), _ch(transb), ip(ms), ip(ns), ip(ks),
                                    float(alpha), _ptr_array(As), ip(ldas), _ptr_array(Bs),
                                    ip(ldbs), float(beta), _ptr_array(Cs), ip(ldcs), batch,
                                    ip(info), int(nthreads))
    if r != 0:
        raise ValueError("oracle_dgemm_vbatched: status %d" % r)
    return info


def _zptr(a: np.ndarray) -> int:
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    return a.ctypes.data


def _pair(z):
    z = complex(z)
    return (ctypes.c_double * 2)(z.real, z.imag)


def zgemm(transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc) -> int:
    """One complex instance on C-contiguous complex128 buffers (interleaved
    real / imaginary binary64 pairs); C is updated in place.  Returns 0 or
    -(argument number)."""
    r = lib().oracle_zgemm(_ch(transa), _ch(transb), m, n, k, _pair(alpha), _zptr(A), lda,
                           _zptr(B), ldb, _pair(beta), _zptr(C), ldc)
    if r == -100:
        raise MemoryError("oracle_zgemm: allocation failed")
    return r


def zgemm_batched(transa, transb, m, n, k, alpha, A, B, beta, C, nthreads=0):
    """Uniform complex batch: A, B, C are (batch, cols, ld) complex128 arrays
    (ld in complex elements); C is updated in place."""
    As, Bs, Cs = _split(A), _split(B), _split(C)
    batch = len(Cs)
    assert len(As) == batch and len(Bs) == batch
    ta, tb = transa in "TtCc", transb in "TtCc"
    lda = As[0].shape[-1] if batch else max(1, k if ta else m)
    ldb = Bs[0].shape[-1] if batch else max(1, n if tb else k)
    ldc = Cs[0].shape[-1] if batch else max(1, m)
    arr = lambda ms: (ctypes.c_void_p * len(ms))(*[_zptr(a) for a in ms])
    r = lib().oracle_zgemm_batched(_ch(transa), _ch(transb), m, n, k, _pair(alpha), arr(As),
                                   lda, arr(Bs), ldb, _pair(beta), arr(Cs), ldc, batch,
                                   int(nthreads))
    if r != 0:
        raise ValueError("oracle_zgemm_batched: info %d" % r)
