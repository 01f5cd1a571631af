"""Python binding of the bgemm C ABI (include/bgemm.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libbgemm.so``.  Torch is used for device memory and the current
stream.  If the library is missing, importing works but every call raises
``RuntimeError``; there is no fallback path.

Matrix convention: a batch of column-major matrices (rows x cols, leading
dimension ld) is a CUDA float64 tensor of shape (batch, cols, ld), or a list
of (cols, ld) tensors; element (r, c) of instance b is ``t[b, c, r]``.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbgemm.so")
_lib = None

STATUS = {0: "SUCCESS", 1: "INVALID_VALUE", 2: "NOT_SUPPORTED", 3: "DEVICE_ERROR",
          4: "ALLOC_FAILED", 5: "INVALID_HANDLE", 6: "WORKSPACE_TOO_SMALL"}

# every symbol include/bgemm.h declares
EXPORTS = ["bg_version", "bg_status_string", "bg_create", "bg_destroy", "bg_set_stream",
           "bg_get_stream", "bg_set_workspace", "bg_workspace_bytes_needed",
           "bg_last_invalid_arg", "bg_check_batched_args", "bg_dgemm_batched",
           "bg_dgemm_vbatched", "bg_set_uniform_class", "bg_gemm_batched_mode",
           "bg_zgemm_batched", "bg_zgate2_batched", "bg_noalloc_max_batch",
           "bg_dgemm_vbatched_noalloc"]

# bg_mode_t
MODE_FP64, MODE_FP32, MODE_BF16, MODE_EMU, MODE_EMU_I8, MODE_EMU_F32 = 0, 1, 2, 3, 4, 5
MODES = {"fp64": MODE_FP64, "fp32": MODE_FP32, "bf16": MODE_BF16, "emu": MODE_EMU,
         "i8emu": MODE_EMU_I8, "f32emu": MODE_EMU_F32}


class BgemmError(RuntimeError):
    def __init__(self, fn, status, arg=0):
        self.status = status
        self.arg = arg
        msg = "%s: %s" % (fn, STATUS.get(status, str(status)))
        if arg:
            msg += " (argument %d)" % arg
        super().__init__(msg)


def lib(path: str | None = None):
    """Loads libbgemm.so (raises if it has not been built).  ``path``, or else
    the environment variable BG_LIB, selects another build of the same
    interface (e.g. a tuning variant); it must be given before the first
    call."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("BG_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libbgemm.so not built: run python -m paper_2203_09353_amd.build")
    L = ctypes.CDLL(path)
    vp, i, d, c = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_char
    L.bg_version.restype = i
    L.bg_version.argtypes = []
    L.bg_status_string.restype = ctypes.c_char_p
    L.bg_status_string.argtypes = [i]
    L.bg_create.restype = i
    L.bg_create.argtypes = [ctypes.POINTER(vp)]
    L.bg_destroy.restype = i
    L.bg_destroy.argtypes = [vp]
    L.bg_set_stream.restype = i
    L.bg_set_stream.argtypes = [vp, vp]
    L.bg_get_stream.restype = i
    L.bg_get_stream.argtypes = [vp, ctypes.POINTER(vp)]
    L.bg_set_workspace.restype = i
    L.bg_set_workspace.argtypes = [vp, ctypes.c_ulonglong]
    L.bg_workspace_bytes_needed.restype = ctypes.c_ulonglong
    L.bg_workspace_bytes_needed.argtypes = [i]
    L.bg_last_invalid_arg.restype = i
    L.bg_last_invalid_arg.argtypes = [vp]
    L.bg_check_batched_args.restype = i
    L.bg_check_batched_args.argtypes = [c, c, i, i, i, vp, i, vp, i, vp, i, i]
    L.bg_dgemm_batched.restype = i
    L.bg_dgemm_batched.argtypes = [vp, c, c, i, i, i, d, vp, i, vp, i, d, vp, i, i]
    L.bg_dgemm_vbatched.restype = i
    L.bg_dgemm_vbatched.argtypes = [vp, c, c, vp, vp, vp, d, vp, vp, vp, vp, d, vp, vp, i, vp]
    L.bg_set_uniform_class.restype = i
    L.bg_set_uniform_class.argtypes = [vp, i]
    dp2 = ctypes.POINTER(ctypes.c_double)
    L.bg_zgemm_batched.restype = i
    L.bg_zgemm_batched.argtypes = [vp, c, c, i, i, i, dp2, vp, i, vp, i, dp2, vp, i, i]
    L.bg_zgate2_batched.restype = i
    L.bg_zgate2_batched.argtypes = [vp, i, vp, vp, vp, i, vp]
    L.bg_gemm_batched_mode.restype = i
    L.bg_gemm_batched_mode.argtypes = [vp, i, i, c, c, i, i, i, d, vp, i, vp, i, d, vp, i, i]
    L.bg_noalloc_max_batch.restype = i
    L.bg_noalloc_max_batch.argtypes = []
    L.bg_dgemm_vbatched_noalloc.restype = i
    L.bg_dgemm_vbatched_noalloc.argtypes = [vp, c, c, vp, vp, vp, d, vp, vp, vp, vp, d, vp, vp, i,
                                            vp, ctypes.POINTER(i)]
    _lib = L
    return L


def _ch(t):
    return t.encode()[:1] if t else b"\0"


def check_batched_args(transa, transb, m, n, k, A, lda, B, ldb, C, ldc, batch) -> int:
    """Host-only argument check (no device); 0 or the bad argument's number."""
    return lib().bg_check_batched_args(_ch(transa), _ch(transb), m, n, k, A, lda, B, ldb, C,
                                       ldc, batch)


def dgemm_vbatched_noalloc_raw(transa, transb, pm, pn, pk, alpha, pA, plda, pB, pldb, beta, pC,
                               pldc, batch, pinfo):
    """bg_dgemm_vbatched_noalloc on torch's current stream of the current
    device; returns (status, bad argument number)."""
    bad = ctypes.c_int(-1)
    st = lib().bg_dgemm_vbatched_noalloc(torch.cuda.current_stream().cuda_stream, _ch(transa),
                                         _ch(transb), pm, pn, pk, float(alpha), pA, plda, pB,
                                         pldb, float(beta), pC, pldc, batch, pinfo,
                                         ctypes.byref(bad))
    return st, bad.value


def pointer_array(x) -> torch.Tensor:
    """Device int64 tensor of per-instance data pointers for a (batch, cols,
    ld) tensor or a list of tensors (kept alive by the caller)."""
    if isinstance(x, torch.Tensor):
        assert x.dim() == 3 and x.dtype in (torch.float64, torch.complex128) and x.is_cuda
        nb = x.shape[0]
        base = x.data_ptr()
        step = x.stride(0) * x.element_size()
        return torch.arange(nb, dtype=torch.int64, device=x.device) * step + base
    ptrs = [t.data_ptr() for t in x]
    dev = x[0].device if len(x) else torch.device("cuda")
    return torch.tensor(ptrs, dtype=torch.int64, device=dev)


class Handle:
    """A bgemm handle on the current device, enqueuing on torch's current
    stream at each call."""

    def __init__(self, workspace_bytes: int | None = None):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.bg_create(ctypes.byref(h))
        if st != 0:
            raise BgemmError("bg_create", st)
        self._h = h
        if workspace_bytes:
            self.set_workspace(workspace_bytes)

    def close(self):
        if getattr(self, "_h", None):
            self._L.bg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        self._L.bg_set_stream(self._h, torch.cuda.current_stream().cuda_stream)

    def set_workspace(self, nbytes: int):
        st = self._L.bg_set_workspace(self._h, int(nbytes))
        if st != 0:
            raise BgemmError("bg_set_workspace", st)

    def set_uniform_class(self, cls: int):
        st = self._L.bg_set_uniform_class(self._h, int(cls))
        if st != 0:
            raise BgemmError("bg_set_uniform_class", st)

    def last_invalid_arg(self) -> int:
        return self._L.bg_last_invalid_arg(self._h)

    # raw entry points: pointer arrays and sizes as given --------------------
    def dgemm_batched_raw(self, transa, transb, m, n, k, alpha, pA, lda, pB, ldb, beta, pC, ldc,
                          batch) -> int:
        self._sync_stream()
        return self._L.bg_dgemm_batched(self._h, _ch(transa), _ch(transb), m, n, k, float(alpha),
                                        pA, lda, pB, ldb, float(beta), pC, ldc, batch)

    def gemm_batched_mode_raw(self, mode, slices, transa, transb, m, n, k, alpha, pA, lda, pB,
                              ldb, beta, pC, ldc, batch) -> int:
        self._sync_stream()
        return self._L.bg_gemm_batched_mode(self._h, int(mode), int(slices), _ch(transa),
                                            _ch(transb), m, n, k, float(alpha), pA, lda, pB, ldb,
                                            float(beta), pC, ldc, batch)

    def zgemm_batched_raw(self, transa, transb, m, n, k, alpha, pA, lda, pB, ldb, beta, pC, ldc,
                          batch) -> int:
        self._sync_stream()
        al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
        return self._L.bg_zgemm_batched(self._h, _ch(transa), _ch(transb), m, n, k, al, pA, lda,
                                        pB, ldb, be, pC, ldc, batch)

    def zbatched(self, A, B, C, m, n, k, alpha=1.0, beta=0.0, transa="N", transb="N",
                 ptrs=None):
        """Complex batch on stacked (batch, cols, ld) complex128 CUDA tensors
        (or lists of (cols, ld) tensors); ld in complex elements."""
        a0, b0, c0 = A[0], B[0], C[0]
        lda, ldb, ldc = a0.shape[-1], b0.shape[-1], c0.shape[-1]
        batch = C.shape[0] if isinstance(C, torch.Tensor) else len(C)
        if ptrs is None:
            ptrs = (pointer_array(A), pointer_array(B), pointer_array(C))
        pA, pB, pC = ptrs
        st = self.zgemm_batched_raw(transa, transb, m, n, k, alpha, pA.data_ptr(), lda,
                                    pB.data_ptr(), ldb, beta, pC.data_ptr(), ldc, batch)
        if st != 0:
            raise BgemmError("bg_zgemm_batched", st, self.last_invalid_arg())
        return ptrs

    def zgate2(self, S, sites, U, psi, info=None):
        """Two-spin gates in place: sites a CUDA int32 tensor (batch,), U a
        CUDA complex128 tensor (batch, 4, 4) of ordinary matrices, psi a CUDA
        complex128 tensor (batch, 2^S).  Returns the info tensor."""
        batch = psi.shape[0]
        Ucm = U.transpose(1, 2).contiguous()        # column-major storage
        pU = (torch.arange(batch, device=psi.device, dtype=torch.int64) * 256 + Ucm.data_ptr())
        pP = (torch.arange(batch, device=psi.device, dtype=torch.int64) * (psi.stride(0) * 16)
              + psi.data_ptr())
        sites = sites.to(device=psi.device, dtype=torch.int32).contiguous()
        if info is None:
            info = torch.empty(batch, dtype=torch.int32, device=psi.device)
        self._sync_stream()
        st = self._L.bg_zgate2_batched(self._h, int(S), sites.data_ptr(), pU.data_ptr(),
                                       pP.data_ptr(), batch, info.data_ptr())
        if st != 0:
            raise BgemmError("bg_zgate2_batched", st, self.last_invalid_arg())
        self._keep = (Ucm, pU, pP, sites)
        return info

    def dgemm_vbatched_raw(self, transa, transb, pm, pn, pk, alpha, pA, plda, pB, pldb, beta, pC,
                           pldc, batch, pinfo) -> int:
        self._sync_stream()
        return self._L.bg_dgemm_vbatched(self._h, _ch(transa), _ch(transb), pm, pn, pk,
                                         float(alpha), pA, plda, pB, pldb, float(beta), pC, pldc,
                                         batch, pinfo)

    # tensor-level helpers ------------------------------------------------------
    def batched(self, A, B, C, m, n, k, alpha=1.0, beta=0.0, transa="N", transb="N",
                ptrs=None):
        """C <- alpha op(A) op(B) + beta C for stacked (batch, cols, ld) CUDA
        tensors or lists of (cols, ld) tensors; the leading dimensions are read
        from the last axis.  ``ptrs`` may pass precomputed (pA, pB, pC)
        pointer tensors.  Returns the pointer tensors."""
        a0, b0, c0 = A[0], B[0], C[0]
        lda, ldb, ldc = a0.shape[-1], b0.shape[-1], c0.shape[-1]
        batch = C.shape[0] if isinstance(C, torch.Tensor) else len(C)
        if ptrs is None:
            ptrs = (pointer_array(A), pointer_array(B), pointer_array(C))
        pA, pB, pC = ptrs
        st = self.dgemm_batched_raw(transa, transb, m, n, k, alpha, pA.data_ptr(), lda,
                                    pB.data_ptr(), ldb, beta, pC.data_ptr(), ldc, batch)
        if st != 0:
            raise BgemmError("bg_dgemm_batched", st, self.last_invalid_arg())
        return ptrs

    def batched_mode(self, mode, A, B, C, m, n, k, alpha=1.0, beta=0.0, slices=0, transa="N",
                     transb="N", ptrs=None):
        """As ``batched`` in precision mode ``mode`` ("fp64", "fp32", "bf16",
        "emu", "i8emu", "f32emu" or a bg_mode_t value); ``slices`` is an emulated
        mode's digit slice count (1..8)."""
        mode = MODES.get(mode, mode) if isinstance(mode, str) else mode
        if isinstance(mode, str):
            raise ValueError("unknown mode " + mode)
        a0, b0, c0 = A[0], B[0], C[0]
        lda, ldb, ldc = a0.shape[-1], b0.shape[-1], c0.shape[-1]
        batch = C.shape[0] if isinstance(C, torch.Tensor) else len(C)
        if ptrs is None:
            ptrs = (pointer_array(A), pointer_array(B), pointer_array(C))
        pA, pB, pC = ptrs
        st = self.gemm_batched_mode_raw(mode, slices, transa, transb, m, n, k, alpha,
                                        pA.data_ptr(), lda, pB.data_ptr(), ldb, beta,
                                        pC.data_ptr(), ldc, batch)
        if st != 0:
            raise BgemmError("bg_gemm_batched_mode", st, self.last_invalid_arg())
        return ptrs

    def vbatched(self, As, Bs, Cs, ms, ns, ks, alpha=1.0, beta=0.0, transa="N", transb="N",
                 ldas=None, ldbs=None, ldcs=None, info=None, ptrs=None):
        """Variable sizes; As, Bs, Cs are lists of (cols, ld) CUDA tensors (or
        ``ptrs`` = (pA, pB, pC) device pointer tensors).  ms, ns, ks (and the
        ld arrays) are CUDA int32 tensors or sequences.  Returns the device
        info tensor (int32)."""
        dev = torch.device("cuda", torch.cuda.current_device())

        def ivec(x):
            if isinstance(x, torch.Tensor):
                return x.to(device=dev, dtype=torch.int32).contiguous()
            return torch.tensor(list(x), dtype=torch.int32, device=dev)

        batch = len(ms)
        ldas = ivec([a.shape[-1] for a in As] if ldas is None else ldas)
        ldbs = ivec([b.shape[-1] for b in Bs] if ldbs is None else ldbs)
        ldcs = ivec([c.shape[-1] for c in Cs] if ldcs is None else ldcs)
        ms, ns, ks = ivec(ms), ivec(ns), ivec(ks)
        if info is None:
            info = torch.empty(batch, dtype=torch.int32, device=dev)
        if ptrs is None:
            ptrs = (pointer_array(As), pointer_array(Bs), pointer_array(Cs))
        pA, pB, pC = ptrs
        st = self.dgemm_vbatched_raw(transa, transb, ms.data_ptr(), ns.data_ptr(), ks.data_ptr(),
                                     alpha, pA.data_ptr(), ldas.data_ptr(), pB.data_ptr(),
                                     ldbs.data_ptr(), beta, pC.data_ptr(), ldcs.data_ptr(),
                                     batch, info.data_ptr())
        if st != 0:
            raise BgemmError("bg_dgemm_vbatched", st, self.last_invalid_arg())
        return info
