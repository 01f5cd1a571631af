// Two-spin gates on batches of S-spin states (the paper's Monte Carlo step
// applies a local unitary to a random pair of neighbouring spins before the
// entropy product, Section III, Alg. 1).  Amplitude x of a state has spin j in
// bit j; a gate U (4 x 4 complex, column-major, interleaved binary64 pairs)
// on spins (s, s + 1) maps every quadruple of amplitudes differing only in
// those bits, local index q = b_s + 2 b_{s+1}, to U times itself.
//
// The operation streams each state through once (64 bytes read and written
// per quadruple, 16 complex multiply-adds): HBM-bound, so one thread per
// quadruple with 16-byte loads and stores, the gate in scalar registers, and
// consecutive threads on consecutive quadruples (coalesced for every s).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bgemm_internal.h"

namespace bg {

typedef double gd2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_gate2(int S, const int* __restrict__ sites,
                                               const double* const* __restrict__ Up,
                                               double* const* __restrict__ Psi, int batch,
                                               int* __restrict__ info) {
  const int64_t quads = (int64_t)1 << (S - 2);
  for (int inst = blockIdx.y; inst < batch; inst += gridDim.y) {
    const int s = sites[inst];
    const bool ok = s >= 0 && s <= S - 2;
    if (info && blockIdx.x == 0 && threadIdx.x == 0) info[inst] = ok ? 0 : -3;
    if (!ok) continue;
    const double* U = Up[inst];
    double ur[16], ui[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      ur[e] = U[2 * e];
      ui[e] = U[2 * e + 1];
    }
    double* psi = Psi[inst];
    const bool vec = ((uintptr_t)psi & 15) == 0;
    const int64_t lowmask = ((int64_t)1 << s) - 1;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < quads;
         g += (int64_t)gridDim.x * 256) {
      const int64_t x0 = (g & lowmask) | ((g >> s) << (s + 2));
      int64_t x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = x0 + ((int64_t)(q & 1) << s) + ((int64_t)(q >> 1) << (s + 1));
      double vr[4], vi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (vec) {
          const gd2 v = *(const gd2*)(psi + 2 * x[q]);
          vr[q] = v.x;
          vi[q] = v.y;
        } else {
          vr[q] = psi[2 * x[q]];
          vi[q] = psi[2 * x[q] + 1];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int qp = 0; qp < 4; ++qp) {
          const double a = ur[4 * qp + q], b = ui[4 * qp + q];
          ar += a * vr[qp] - b * vi[qp];
          ai += a * vi[qp] + b * vr[qp];
        }
        if (vec) {
          *(gd2*)(psi + 2 * x[q]) = gd2{ar, ai};
        } else {
          psi[2 * x[q]] = ar;
          psi[2 * x[q] + 1] = ai;
        }
      }
    }
  }
}

hipError_t launch_gate2(int S, const int* sites, const double* const* U, double* const* psi,
                        int batch, int* info, hipStream_t s) {
  const int64_t quads = (int64_t)1 << (S - 2);
  const int64_t gx = (quads + 255) / 256;
  const unsigned bx = (unsigned)(gx < 4096 ? gx : 4096);
  const unsigned by = (unsigned)(batch < 65535 ? batch : 65535);
  hipLaunchKernelGGL(k_gate2, dim3(bx, by), dim3(256), 0, s, S, sites, U, psi, batch, info);
  return hipGetLastError();
}

}  // namespace bg
