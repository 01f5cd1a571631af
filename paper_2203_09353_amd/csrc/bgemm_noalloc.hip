// Variable-size batch without a handle and without any allocation: the
// planner's buffers (per-class prefix sums, block sums, queue heads and the
// tile -> instance map) live in one library-owned array of device memory per
// GPU instead of a handle's workspace.  The kernels are those of
// bg_dgemm_vbatched.
#include <mutex>

#include "../../include/bgemm.h"
#include "bgemm_internal.h"

namespace {

// The planner's buffers.  Each GPU the library runs on holds its own copy
// until the process ends; every call on that GPU reuses it.
static __device__ __align__(256) unsigned char scratch[BG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
  void* ptr = nullptr;   // device address of `scratch` on this device
  int num_cus = 0;
  bool ready = false;
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// Looks up the device address of `scratch` (and the CU count) once per
// device, with that device current.  In host code the array's name is only a
// stand-in for the symbol, never a device address, so every use below goes
// through the looked-up pointer.
hipError_t device_scratch(int dev, DeviceScratch* out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (!d.ready) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    d.ptr = p;
    d.num_cus = cus > 0 ? cus : 1;
    d.ready = true;
  }
  *out = d;
  return hipSuccess;
}

}  // namespace

extern "C" {

int bg_noalloc_max_batch(void) {
  // largest batch whose planning buffers fit the array (the map is optional)
  int lo = 0, hi = 1 << 30;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (bg::vbatched_workspace_bytes(mid) <= (size_t)BG_NOALLOC_SCRATCH_BYTES) lo = mid;
    else hi = mid;
  }
  return lo;
}

bg_status_t bg_dgemm_vbatched_noalloc(void* stream, char transa, char transb, const int* d_m,
                                      const int* d_n, const int* d_k, double alpha,
                                      const double* const* dA, const int* d_lda,
                                      const double* const* dB, const int* d_ldb, double beta,
                                      double* const* dC, const int* d_ldc, int batch,
                                      int* d_info, int* bad_arg) {
  const int bad = bg::vbatched_host_args(transa, transb, d_m, d_n, d_k, dA, d_lda, dB, d_ldb, dC,
                                         d_ldc, batch);
  if (bad_arg) *bad_arg = bad;
  if (bad) return BG_STATUS_INVALID_VALUE;
  if (batch == 0) return BG_STATUS_SUCCESS;
  if (bg::vbatched_workspace_bytes(batch) > (size_t)BG_NOALLOC_SCRATCH_BYTES)
    return BG_STATUS_WORKSPACE_TOO_SMALL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
  DeviceScratch d;
  if (device_scratch(dev, &d) != hipSuccess) return BG_STATUS_DEVICE_ERROR;
  const bg::VbatchedArgs a = bg::vbatched_args(transa, transb, d_m, d_n, d_k, alpha, dA, d_lda, dB,
                                               d_ldb, beta, dC, d_ldc, batch, d_info);
  const bg::VbWorkspace ws{d.ptr, (size_t)BG_NOALLOC_SCRATCH_BYTES};
  const hipError_t e = bg::launch_vbatched(a, ws, d.num_cus, (hipStream_t)stream);
  return e == hipSuccess ? BG_STATUS_SUCCESS : BG_STATUS_DEVICE_ERROR;
}

}  // extern "C"
