// C-ABI layer: handle, argument rules, quick returns and dispatch to the
// kernel launchers.  Host code only; everything here runs before a launch.
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "../../include/bgemm.h"
#include "bgemm_internal.h"

struct bg_handle {
  unsigned magic;
  int device;
  int num_cus;
  hipStream_t stream;
  void* ws;
  size_t ws_bytes;
  int last_invalid_arg;
  int force_class;
};

static const unsigned kMagic = 0xB6E11A5Du;

static bool valid(bg_handle_t h) { return h != nullptr && h->magic == kMagic; }

static int trans_code(char t) {
  if (t == 'N' || t == 'n') return 0;
  if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
  return -1;
}

static int imax1(int a) { return a > 1 ? a : 1; }

// Makes the handle's device current for the duration of a call and restores
// the caller's device afterwards.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

namespace bg {

// Host-side rules of the variable-size call (sizes are checked on the
// device); returns the argument number of the first bad argument, else 0.
int vbatched_host_args(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
                       const void* dA, const int* d_lda, const void* dB, const int* d_ldb,
                       const void* dC, const int* d_ldc, int batch) {
  if (trans_code(transa) < 0) return 1;
  if (trans_code(transb) < 0) return 2;
  if (batch < 0) return 14;
  if (batch > 0) {
    if (!d_m) return 3;
    if (!d_n) return 4;
    if (!d_k) return 5;
    if (!dA) return 7;
    if (!d_lda) return 8;
    if (!dB) return 9;
    if (!d_ldb) return 10;
    if (!dC) return 12;
    if (!d_ldc) return 13;
  }
  return 0;
}

VbatchedArgs vbatched_args(char transa, char transb, const int* d_m, const int* d_n,
                           const int* d_k, double alpha, const double* const* dA,
                           const int* d_lda, const double* const* dB, const int* d_ldb,
                           double beta, double* const* dC, const int* d_ldc, int batch,
                           int* d_info) {
  VbatchedArgs a;
  a.ta = trans_code(transa) == 1; a.tb = trans_code(transb) == 1;
  a.m = d_m; a.n = d_n; a.k = d_k;
  a.alpha = alpha; a.beta = beta;
  a.A = dA; a.lda = d_lda; a.B = dB; a.ldb = d_ldb; a.C = dC; a.ldc = d_ldc;
  a.batch = batch; a.info = d_info;
  return a;
}

}  // namespace bg

extern "C" {

int bg_version(void) { return 100; }

const char* bg_status_string(bg_status_t s) {
  switch (s) {
    case BG_STATUS_SUCCESS: return "BG_STATUS_SUCCESS";
    case BG_STATUS_INVALID_VALUE: return "BG_STATUS_INVALID_VALUE";
    case BG_STATUS_NOT_SUPPORTED: return "BG_STATUS_NOT_SUPPORTED";
    case BG_STATUS_DEVICE_ERROR: return "BG_STATUS_DEVICE_ERROR";
    case BG_STATUS_ALLOC_FAILED: return "BG_STATUS_ALLOC_FAILED";
    case BG_STATUS_INVALID_HANDLE: return "BG_STATUS_INVALID_HANDLE";
    case BG_STATUS_WORKSPACE_TOO_SMALL: return "BG_STATUS_WORKSPACE_TOO_SMALL";
  }
  return "BG_STATUS_UNKNOWN";
}

static size_t default_ws_bytes() {
  const char* e = getenv("BG_WORKSPACE_MB");
  if (e && *e) {
    long v = strtol(e, nullptr, 10);
    if (v > 0) return (size_t)v << 20;
  }
  return (size_t)BG_DEFAULT_WORKSPACE_BYTES;
}

bg_status_t bg_create(bg_handle_t* out) {
  if (!out) return BG_STATUS_INVALID_VALUE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return BG_STATUS_DEVICE_ERROR;
  bg_handle* h = (bg_handle*)calloc(1, sizeof(bg_handle));
  if (!h) return BG_STATUS_ALLOC_FAILED;
  h->magic = kMagic;
  h->device = dev;
  h->num_cus = cus > 0 ? cus : 1;
  h->stream = nullptr;
  h->force_class = -1;
  h->ws_bytes = default_ws_bytes();
  if (hipMalloc(&h->ws, h->ws_bytes) != hipSuccess) {
    free(h);
    return BG_STATUS_ALLOC_FAILED;
  }
  *out = h;
  return BG_STATUS_SUCCESS;
}

bg_status_t bg_destroy(bg_handle_t h) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  h->magic = 0;
  free(h);
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bg_set_stream(bg_handle_t h, void* stream) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  h->stream = (hipStream_t)stream;
  return BG_STATUS_SUCCESS;
}

bg_status_t bg_get_stream(bg_handle_t h, void** stream) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  if (!stream) return BG_STATUS_INVALID_VALUE;
  *stream = (void*)h->stream;
  return BG_STATUS_SUCCESS;
}

unsigned long long bg_workspace_bytes_needed(int batch) {
  return batch <= 0 ? 0ull : (unsigned long long)bg::vbatched_workspace_bytes(batch);
}

bg_status_t bg_set_workspace(bg_handle_t h, unsigned long long bytes) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  if (bytes == 0) return BG_STATUS_INVALID_VALUE;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)bytes) != hipSuccess) return BG_STATUS_ALLOC_FAILED;
  if (h->ws) (void)hipFree(h->ws);
  h->ws = p;
  h->ws_bytes = (size_t)bytes;
  return BG_STATUS_SUCCESS;
}

int bg_last_invalid_arg(bg_handle_t h) { return valid(h) ? h->last_invalid_arg : 0; }

bg_status_t bg_set_uniform_class(bg_handle_t h, int cls) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  if (cls < -1 || cls >= bg::TC_COUNT) return BG_STATUS_INVALID_VALUE;
  h->force_class = cls;
  return BG_STATUS_SUCCESS;
}

int bg_check_batched_args(char transa, char transb, int m, int n, int k, const void* dA, int lda,
                          const void* dB, int ldb, const void* dC, int ldc, int batch) {
  const int ta = trans_code(transa), tb = trans_code(transb);
  if (ta < 0) return 1;
  if (tb < 0) return 2;
  if (m < 0) return 3;
  if (n < 0) return 4;
  if (k < 0) return 5;
  if (lda < imax1(ta ? k : m)) return 8;
  if (ldb < imax1(tb ? n : k)) return 10;
  if (ldc < imax1(m)) return 13;
  if (batch < 0) return 14;
  // Pointer arrays are required only when the call will read them.
  if (batch > 0 && m > 0 && n > 0) {
    if (!dC) return 12;
    if (k > 0) {
      if (!dA) return 7;
      if (!dB) return 9;
    }
  }
  return 0;
}

bg_status_t bg_dgemm_batched(bg_handle_t h, char transa, char transb, int m, int n, int k,
                             double alpha, const double* const* dA, int lda,
                             const double* const* dB, int ldb, double beta, double* const* dC,
                             int ldc, int batch) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  const int bad = bg_check_batched_args(transa, transb, m, n, k, dA, lda, dB, ldb, dC, ldc, batch);
  h->last_invalid_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0 || m == 0 || n == 0) return BG_STATUS_SUCCESS;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (no_product && beta == 1.0) return BG_STATUS_SUCCESS;
  DeviceGuard guard(h->device);
  if (!guard.ok) return BG_STATUS_DEVICE_ERROR;
  hipError_t e;
  if (no_product) {
    e = bg::launch_scale(beta, dC, ldc, m, n, batch, h->stream);
  } else {
    bg::UniformArgs a;
    a.ta = trans_code(transa) == 1;
    a.tb = trans_code(transb) == 1;
    a.m = m; a.n = n; a.k = k;
    a.alpha = alpha; a.beta = beta;
    a.A = dA; a.lda = lda; a.B = dB; a.ldb = ldb; a.C = dC; a.ldc = ldc;
    a.batch = batch;
    a.num_cus = h->num_cus;
    a.ws = h->ws;
    a.ws_bytes = h->ws_bytes;
    const bg::TileClass cls = bg::pick_uniform_class(m, n, k, batch, h->num_cus, h->force_class);
    e = bg::launch_uniform(a, cls, h->stream);
    if (e == hipErrorInvalidValue) return BG_STATUS_NOT_SUPPORTED;
  }
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bg_gemm_batched_mode(bg_handle_t h, int mode, int slices, char transa, char transb,
                                 int m, int n, int k, double alpha, const double* const* dA,
                                 int lda, const double* const* dB, int ldb, double beta,
                                 double* const* dC, int ldc, int batch) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  if (mode == BG_MODE_FP64)
    return bg_dgemm_batched(h, transa, transb, m, n, k, alpha, dA, lda, dB, ldb, beta, dC, ldc,
                            batch);
  int bad = 0;
  const bool sliced = mode == BG_MODE_EMU || mode == BG_MODE_EMU_I8 || mode == BG_MODE_EMU_F32;
  if (mode != BG_MODE_FP32 && mode != BG_MODE_BF16 && !sliced)
    bad = 101;
  else if (sliced && (slices < 1 || slices > 8))
    bad = 102;
  else bad = bg_check_batched_args(transa, transb, m, n, k, dA, lda, dB, ldb, dC, ldc, batch);
  h->last_invalid_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0 || m == 0 || n == 0) return BG_STATUS_SUCCESS;
  const bool no_product = (alpha == 0.0 || k == 0);
  if (no_product && beta == 1.0) return BG_STATUS_SUCCESS;
  if (!no_product && (trans_code(transa) != 0 || trans_code(transb) != 0))
    return BG_STATUS_NOT_SUPPORTED;
  DeviceGuard guard(h->device);
  if (!guard.ok) return BG_STATUS_DEVICE_ERROR;
  hipError_t e;
  if (no_product) {
    e = bg::launch_scale(beta, dC, ldc, m, n, batch, h->stream);
  } else {
    bg::UniformArgs a;
    a.ta = false; a.tb = false;
    a.m = m; a.n = n; a.k = k;
    a.alpha = alpha; a.beta = beta;
    a.A = dA; a.lda = lda; a.B = dB; a.ldb = ldb; a.C = dC; a.ldc = ldc;
    a.batch = batch;
    if (mode == BG_MODE_EMU_I8) {
      // exact int32 diagonal sums need k <= 8192; the exponents of at least
      // one instance must fit the workspace
      if (k > 8192) return BG_STATUS_NOT_SUPPORTED;
      if (h->ws_bytes < (size_t)(m + n) * sizeof(int)) return BG_STATUS_ALLOC_FAILED;
      e = bg::launch_emu8(a, slices, h->ws, h->ws_bytes, h->stream);
    } else {
      e = bg::launch_uniform_lowp(a, mode, slices, h->stream);
    }
    if (e == hipErrorInvalidValue) return BG_STATUS_NOT_SUPPORTED;
  }
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

static int ztrans(char t) {
  if (t == 'N' || t == 'n') return 0;
  if (t == 'T' || t == 't') return 1;
  if (t == 'C' || t == 'c') return 2;
  return -1;
}

bg_status_t bg_zgemm_batched(bg_handle_t h, char transa, char transb, int m, int n, int k,
                             const double* alpha, const double* const* dA, int lda,
                             const double* const* dB, int ldb, const double* beta,
                             double* const* dC, int ldc, int batch) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  int bad = bg_check_batched_args(transa, transb, m, n, k, dA, lda, dB, ldb, dC, ldc, batch);
  if (!bad && !alpha) bad = 6;
  if (!bad && !beta) bad = 11;
  h->last_invalid_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0 || m == 0 || n == 0) return BG_STATUS_SUCCESS;
  const bool no_product = (alpha[0] == 0.0 && alpha[1] == 0.0) || k == 0;
  const bool beta_one = beta[0] == 1.0 && beta[1] == 0.0;
  if (no_product && beta_one) return BG_STATUS_SUCCESS;
  DeviceGuard guard(h->device);
  if (!guard.ok) return BG_STATUS_DEVICE_ERROR;
  hipError_t e;
  if (no_product) {
    e = bg::launch_zscale(beta, dC, ldc, m, n, batch, h->stream);
  } else {
    bg::ZUniformArgs a;
    a.ta = ztrans(transa);
    a.tb = ztrans(transb);
    a.m = m; a.n = n; a.k = k;
    a.alpha = alpha; a.beta = beta;
    a.A = dA; a.lda = lda; a.B = dB; a.ldb = ldb; a.C = dC; a.ldc = ldc;
    a.batch = batch;
    e = bg::launch_zgemm(a, h->stream);
    if (e == hipErrorInvalidValue) return BG_STATUS_NOT_SUPPORTED;
  }
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bg_zgate2_batched(bg_handle_t h, int S, const int* d_site, const double* const* dU,
                              double* const* dPsi, int batch, int* d_info) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  int bad = 0;
  if (S < 2 || S > 40) bad = 2;
  else if (batch > 0 && !d_site) bad = 3;
  else if (batch > 0 && !dU) bad = 4;
  else if (batch > 0 && !dPsi) bad = 5;
  else if (batch < 0) bad = 6;
  h->last_invalid_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0) return BG_STATUS_SUCCESS;
  DeviceGuard guard(h->device);
  if (!guard.ok) return BG_STATUS_DEVICE_ERROR;
  return bg::launch_gate2(S, d_site, dU, dPsi, batch, d_info, h->stream) == hipSuccess
             ? BG_STATUS_SUCCESS
             : BG_STATUS_DEVICE_ERROR;
}

bg_status_t bg_dgemm_vbatched(bg_handle_t h, char transa, char transb, const int* d_m,
                              const int* d_n, const int* d_k, double alpha,
                              const double* const* dA, const int* d_lda, const double* const* dB,
                              const int* d_ldb, double beta, double* const* dC, const int* d_ldc,
                              int batch, int* d_info) {
  if (!valid(h)) return BG_STATUS_INVALID_HANDLE;
  const int bad = bg::vbatched_host_args(transa, transb, d_m, d_n, d_k, dA, d_lda, dB, d_ldb, dC,
                                     d_ldc, batch);
  h->last_invalid_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0) return BG_STATUS_SUCCESS;
  if (bg::vbatched_workspace_bytes(batch) > h->ws_bytes) return BG_STATUS_WORKSPACE_TOO_SMALL;
  DeviceGuard guard(h->device);
  if (!guard.ok) return BG_STATUS_DEVICE_ERROR;
  const bg::VbatchedArgs a = bg::vbatched_args(transa, transb, d_m, d_n, d_k, alpha, dA, d_lda, dB,
                                           d_ldb, beta, dC, d_ldc, batch, d_info);
  bg::VbWorkspace ws{h->ws, h->ws_bytes};
  const hipError_t e = bg::launch_vbatched(a, ws, h->num_cus, h->stream);
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

}  // extern "C"
