// Device side of the request loop: the factor generator (Philox4x64-10,
// Salmon, Moraes, Dror and Shaw, SC'11) and the identity initialiser.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bgemm_internal.h"

namespace bg {

// Philox4x64: round multipliers and Weyl key increments of the published
// definition; ten rounds.
constexpr uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(PHILOX_M0, x[0]), lo0 = PHILOX_M0 * x[0];
    const uint64_t hi1 = __umul64hi(PHILOX_M1, x[2]), lo1 = PHILOX_M1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
}

// Word w -> 2 ((w >> 11) 2^-53) - 1 in [-1, 1) (exact), times scale (one
// rounding).
__device__ __forceinline__ double word_value(uint64_t w, double scale) {
#pragma clang fp contract(off)
  const double u = (double)(w >> 11) * 0x1p-53;
  return (2.0 * u - 1.0) * scale;
}

// Element e of factor (j, client) is word e mod 4 of the block at counter
// (e div 4, j, 0, 0) with key (seed, client).  Each thread makes one block.
__device__ __forceinline__ void fill_job(const FillJob& jb, uint64_t seed, int64_t b0,
                                         int64_t stride) {
  const int64_t total = (int64_t)jb.n * jb.n;
  const int64_t nblk = (total + 3) / 4;
  for (int64_t b = b0; b < nblk; b += stride) {
    uint64_t x[4] = {(uint64_t)b, (uint64_t)jb.j, 0ull, 0ull};
    philox4x64_10(x, seed, (uint64_t)jb.client);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = 4 * b + q;
      if (e < total) jb.out[e] = word_value(x[q], jb.scale);
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_factors(const FillJob* __restrict__ jobs,
                                                      uint64_t seed) {
  const FillJob jb = jobs[blockIdx.y];
  fill_job(jb, seed, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

__global__ __launch_bounds__(256) void k_fill_sweep(const SweepJob* __restrict__ jobs,
                                                    const long long* __restrict__ j0, int t,
                                                    uint64_t seed) {
  const SweepJob sj = jobs[blockIdx.y];
  const FillJob jb{sj.out, j0[sj.client] + t, sj.n, sj.client, sj.scale};
  fill_job(jb, seed, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

__global__ __launch_bounds__(256) void k_advance(long long* __restrict__ j0, int n, int chain) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) j0[i] += chain;
}

__global__ __launch_bounds__(256) void k_fill_one(FillJob jb, uint64_t seed) {
  fill_job(jb, seed, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256);
}

__global__ __launch_bounds__(256) void k_identity(double* __restrict__ out, int n) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256)
    out[e] = (e % (n + 1) == 0) ? 1.0 : 0.0;
}

static unsigned grid_for(int64_t items) {
  const int64_t g = (items + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

hipError_t launch_fill_factors(const FillJob* d_jobs, int njobs, int max_n,
                               unsigned long long seed, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (njobs > 65535 || max_n < 1) return hipErrorInvalidValue;
  const int64_t blocks = ((int64_t)max_n * max_n + 3) / 4;
  hipLaunchKernelGGL(k_fill_factors, dim3(grid_for(blocks), njobs), dim3(256), 0, s, d_jobs,
                     (uint64_t)seed);
  return hipGetLastError();
}

hipError_t launch_fill_sweep(const SweepJob* d_jobs, int njobs, int max_n, const long long* d_j0,
                             int t, unsigned long long seed, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (njobs > 65535 || max_n < 1) return hipErrorInvalidValue;
  const int64_t blocks = ((int64_t)max_n * max_n + 3) / 4;
  hipLaunchKernelGGL(k_fill_sweep, dim3(grid_for(blocks), njobs), dim3(256), 0, s, d_jobs, d_j0, t,
                     (uint64_t)seed);
  return hipGetLastError();
}

hipError_t launch_advance(long long* d_j0, int n, int chain, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(grid_for(n)), dim3(256), 0, s, d_j0, n, chain);
  return hipGetLastError();
}

hipError_t launch_fill_one(double* out, int n, int client, long long j, double scale,
                           unsigned long long seed, hipStream_t s) {
  const FillJob jb{out, j, n, client, scale};
  const int64_t blocks = ((int64_t)n * n + 3) / 4;
  hipLaunchKernelGGL(k_fill_one, dim3(grid_for(blocks)), dim3(256), 0, s, jb, (uint64_t)seed);
  return hipGetLastError();
}

hipError_t launch_identity(double* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_identity, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

}  // namespace bg
