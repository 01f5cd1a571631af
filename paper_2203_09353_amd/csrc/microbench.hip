// Measurement kernels for the roofline denominators and the MFMA lane-layout
// check: attainable FP64 matrix-core and vector throughput, HBM copy/read
// bandwidth, and one FP64 MFMA on caller-supplied fragments.  Built into its
// own library (libbgemm_microbench.so); the GEMM library does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// One v_mfma_f64_16x16x4_f64 by one wave: a[64], b[64] are the per-lane
// source values, c[4*64] the per-lane accumulator (register v of lane l at
// c[4*l + v]), d[4*64] receives the result in the same arrangement.
__global__ void k_mfma_once(const double* a, const double* b, const double* c, double* d) {
  const int l = threadIdx.x;
  d4 acc = {c[4 * l], c[4 * l + 1], c[4 * l + 2], c[4 * l + 3]};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[l], b[l], acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = acc[v];
}

// One v_mfma_f64_4x4x4_4b_f64 (four 4x4x4 blocks) by one wave; a, b, c, d:
// one value per lane.
__global__ void k_mfma4_once(const double* a, const double* b, const double* c, double* d) {
  const int l = threadIdx.x;
  d[l] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[l], b[l], c[l], 0, 0, 0);
}

// One v_mfma_f32_16x16x4_f32: a[64], b[64] per-lane floats, c/d[4*64].
__global__ void k_mfma_f32_once(const float* a, const float* b, const float* c, float* d) {
  const int l = threadIdx.x;
  f4 acc = {c[4 * l], c[4 * l + 1], c[4 * l + 2], c[4 * l + 3]};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l], b[l], acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = acc[v];
}

// One v_mfma_f32_16x16x32_bf16: a/b[8*64] per-lane bfloat16 bit patterns
// (element e of lane l at 8*l + e), c/d[4*64] floats.
__global__ void k_mfma_bf16_once(const unsigned short* a, const unsigned short* b, const float* c,
                                 float* d) {
  const int l = threadIdx.x;
  bf8 va, vb;
  for (int e = 0; e < 8; ++e) {
    unsigned short xa = a[8 * l + e], xb = b[8 * l + e];
    va[e] = __builtin_bit_cast(__bf16, xa);
    vb[e] = __builtin_bit_cast(__bf16, xb);
  }
  f4 acc = {c[4 * l], c[4 * l + 1], c[4 * l + 2], c[4 * l + 3]};
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = acc[v];
}

// One v_mfma_i32_16x16x64_i8: a/b[16*64] per-lane int8 values (element e of
// lane l at 16*l + e, byte e of the lane's 16-byte operand), c/d[4*64] int32.
typedef int i4 __attribute__((ext_vector_type(4)));
__global__ void k_mfma_i8_once(const signed char* a, const signed char* b, const int* c, int* d) {
  const int l = threadIdx.x;
  i4 va, vb;
  for (int w = 0; w < 4; ++w) {
    unsigned ua = 0, ub = 0;
    for (int e = 0; e < 4; ++e) {
      ua |= (unsigned)(unsigned char)a[16 * l + 4 * w + e] << (8 * e);
      ub |= (unsigned)(unsigned char)b[16 * l + 4 * w + e] << (8 * e);
    }
    va[w] = (int)ua;
    vb[w] = (int)ub;
  }
  i4 acc = {c[4 * l], c[4 * l + 1], c[4 * l + 2], c[4 * l + 3]};
  acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(va, vb, acc, 0, 0, 0);
  for (int v = 0; v < 4; ++v) d[4 * l + v] = acc[v];
}

// CHAINS independent accumulators per wave, `iters` rounds of CHAINS MFMAs.
template <int CHAINS>
__global__ __launch_bounds__(256) void k_mfma_peak(double* sink, int iters, double seed) {
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
  d4 acc[CHAINS];
  for (int c = 0; c < CHAINS; ++c) acc[c] = d4{0.0, 0.0, 0.0, (double)c};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
  for (int c = 0; c < CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 1234.5678) sink[threadIdx.x] = s;  // never true in practice; keeps the work
}

// FP64 vector FMA throughput: 8 independent chains per lane.
__global__ __launch_bounds__(256) void k_valu_peak(double* sink, int iters, double seed) {
  double x[8];
  const double m = 1.0 + 1e-12, c = 1e-13;
  for (int i = 0; i < 8; ++i) x[i] = seed + i + threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = __builtin_fma(x[i], m, c);
  }
  double s = 0.0;
  for (int i = 0; i < 8; ++i) s += x[i];
  if (s == 1234.5678) sink[threadIdx.x] = s;
}

// Streaming copy, four 16-byte loads in flight per lane per step.  n2 must be
// a multiple of 4 * gridDim.x * blockDim.x (the host rounds it down).
__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                              int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 3 * stride < n2; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a; dst[i + stride] = b; dst[i + 2 * stride] = c; dst[i + 3 * stride] = d;
  }
}

// Streaming read with a reduction so the loads are kept.
__global__ __launch_bounds__(256) void k_read(const double2* __restrict__ src, int64_t n2, double* sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 3 * stride < n2; i += 4 * stride) {
    const double2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    s += a.x + a.y + b.x + b.y + c.x + c.y + d.x + d.y;
  }
  if (s == 1234.5678) sink[threadIdx.x] = s;
}

// Streaming copy / read, one contiguous chunk of 256 x U 16-byte pairs per
// workgroup (no grid-stride loop): all U loads of a lane are issued before
// the first use, and there are as many workgroups as chunks, so the whole
// device keeps reads in flight.  NT selects nontemporal loads and stores.
// n2 must be a multiple of 256 U (the host rounds it down).
typedef double dv2 __attribute__((ext_vector_type(2)));

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy_chunk(const dv2* __restrict__ src,
                                                    dv2* __restrict__ dst) {
  const int64_t base = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  dv2 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u)
    v[u] = NT ? __builtin_nontemporal_load(src + base + 256 * u) : src[base + 256 * u];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (NT) __builtin_nontemporal_store(v[u], dst + base + 256 * u);
    else dst[base + 256 * u] = v[u];
  }
}

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_read_chunk(const dv2* __restrict__ src, double* sink) {
  const int64_t base = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  double s = 0.0;
  dv2 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u)
    v[u] = NT ? __builtin_nontemporal_load(src + base + 256 * u) : src[base + 256 * u];
#pragma unroll
  for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
  if (s == 1234.5678) sink[threadIdx.x] = s;
}

// 4x4x4 FP64 MFMA (four 4x4 blocks, 512 flop per instruction), 8 chains.
__global__ __launch_bounds__(256) void k_mfma4_peak(double* sink, int iters, double seed) {
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
  double acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = (double)c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
  for (int c = 0; c < 8; ++c) s += acc[c];
  if (s == 1234.5678) sink[threadIdx.x] = s;
}

// int8 matrix core, v_mfma_i32_16x16x64_i8 (32768 operations per
// instruction), 8 independent accumulator chains.
__global__ __launch_bounds__(256) void k_i8_peak(int* sink, int iters, int seed) {
  const int x = seed + (int)threadIdx.x;
  const i4 a = {x, x ^ 0x01010101, x + 7, x * 3};
  const i4 b = {x * 5, x ^ 0x10101010, x - 3, x + 11};
  i4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = i4{c, 0, 0, 0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[c], 0, 0, 0);
  }
  int s = 0;
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 0x12345678) sink[threadIdx.x] = s;
}

static float time_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  hipEventElapsedTime(&ms, a, b);
  return ms;
}

extern "C" {

int mb_mfma_f64_16x16x4(const double* a, const double* b, const double* c, double* d) {
  hipLaunchKernelGGL(k_mfma_once, dim3(1), dim3(64), 0, 0, a, b, c, d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

int mb_mfma_f32_16x16x4(const float* a, const float* b, const float* c, float* d) {
  hipLaunchKernelGGL(k_mfma_f32_once, dim3(1), dim3(64), 0, 0, a, b, c, d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

int mb_mfma_bf16_16x16x32(const unsigned short* a, const unsigned short* b, const float* c,
                          float* d) {
  hipLaunchKernelGGL(k_mfma_bf16_once, dim3(1), dim3(64), 0, 0, a, b, c, d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

int mb_mfma_i8_16x16x64(const signed char* a, const signed char* b, const int* c, int* d) {
  hipLaunchKernelGGL(k_mfma_i8_once, dim3(1), dim3(64), 0, 0, a, b, c, d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

int mb_mfma_f64_4x4x4(const double* a, const double* b, const double* c, double* d) {
  hipLaunchKernelGGL(k_mfma4_once, dim3(1), dim3(64), 0, 0, a, b, c, d);
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

// kind: 0 = MFMA f64 (4 chains), 1 = vector FMA f64, 3 = MFMA f64 with 8
//       chains, 4 = 4x4x4 MFMA f64 with 8 chains.
// Returns the elapsed milliseconds of `reps` launches (negative on error).
double mb_fp64_peak_ms(int kind, int grid, int iters, int reps, double* sink) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&]() {
    if (kind == 0) hipLaunchKernelGGL(k_mfma_peak<4>, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
    else if (kind == 1) hipLaunchKernelGGL(k_valu_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
    else if (kind == 3) hipLaunchKernelGGL(k_mfma_peak<8>, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
    else hipLaunchKernelGGL(k_mfma4_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
  };
  launch();
  hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r) launch();
  hipEventRecord(e1, 0);
  hipError_t err = hipEventSynchronize(e1);
  double ms = err == hipSuccess ? (double)time_ms(e0, e1) : -1.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

// Elapsed milliseconds of `reps` launches of the int8 matrix-core kernel
// (grid workgroups of 256 threads, `iters` rounds), after one warm-up launch.
double mb_i8_peak_ms(int grid, int iters, int reps, int* sink) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  hipLaunchKernelGGL(k_i8_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 3);
  hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_i8_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 3);
  hipEventRecord(e1, 0);
  hipError_t err = hipEventSynchronize(e1);
  double ms = err == hipSuccess ? (double)time_ms(e0, e1) : -1.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

// kind: 0 copy and 1 read with a grid-stride loop over `grid` workgroups;
// 2 copy and 3 read with one 32 KB chunk per workgroup; 4 copy and 5 read
// likewise with nontemporal accesses (`grid` is then ignored).  `bytes` is
// rounded down to whole steps.  Returns the elapsed milliseconds of `reps`
// launches after one warm-up launch (negative on error).
double mb_stream_ms(int kind, const void* src, void* dst, long long bytes, int grid, int reps,
                    double* sink) {
  constexpr int U = 8;
  const bool chunked = kind >= 2;
  const int64_t quad = chunked ? 256ll * U : 4ll * grid * 256;
  const int64_t n2 = (bytes / 16) / quad * quad;
  const int64_t chunks = n2 / (256 * U);
  if (n2 <= 0 || (chunked && chunks > INT32_MAX)) return -1.0;
  const double2* s2 = (const double2*)src;
  double2* d2 = (double2*)dst;
  const dv2* v2s = (const dv2*)src;
  dv2* v2d = (dv2*)dst;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&]() {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, s2, d2, n2); break;
      case 1: hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, 0, s2, n2, sink); break;
      case 2: hipLaunchKernelGGL((k_copy_chunk<U, false>), dim3((unsigned)chunks), dim3(256), 0, 0, v2s, v2d); break;
      case 3: hipLaunchKernelGGL((k_read_chunk<U, false>), dim3((unsigned)chunks), dim3(256), 0, 0, v2s, sink); break;
      case 4: hipLaunchKernelGGL((k_copy_chunk<U, true>), dim3((unsigned)chunks), dim3(256), 0, 0, v2s, v2d); break;
      default: hipLaunchKernelGGL((k_read_chunk<U, true>), dim3((unsigned)chunks), dim3(256), 0, 0, v2s, sink); break;
    }
  };
  launch();
  hipEventRecord(e0, 0);
  for (int r = 0; r < reps; ++r) launch();
  hipEventRecord(e1, 0);
  hipError_t err = hipEventSynchronize(e1);
  double ms = err == hipSuccess ? (double)time_ms(e0, e1) : -1.0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

}  // extern "C"
