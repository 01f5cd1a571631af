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

// One v_mfma_f64_4x4x4_4b_f64 (four 4x4x4 blocks) by one wave with the A
// broadcast controls CBSZ / ABID; a, b, c, d: one value per lane.
template <int CBSZ, int ABID>
__global__ void k_mfma4_once(const double* a, const double* b, const double* c, double* d) {
  const int l = threadIdx.x;
  d[l] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[l], b[l], c[l], CBSZ, ABID, 0);
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

// Half the waves issue MFMA, half issue vector FMA: do the two share the
// FP64 pipeline?
__global__ __launch_bounds__(256) void k_mixed_peak(double* sink, int iters, double seed) {
  const int wave = threadIdx.x >> 6;
  double s = 0.0;
  if (wave & 1) {
    double x[8];
    const double m = 1.0 + 1e-12, c = 1e-13;
    for (int i = 0; i < 8; ++i) x[i] = seed + i + threadIdx.x;
    // 8 FMAs of 128 flop per wave-instruction vs 4 MFMAs of 2048 flop: scale
    // the loop so both halves take about the same time at equal peaks.
    for (int it = 0; it < iters * 8; ++it) {
#pragma unroll
      for (int i = 0; i < 8; ++i) x[i] = __builtin_fma(x[i], m, c);
    }
    for (int i = 0; i < 8; ++i) s += x[i];
  } else {
    const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
    d4 acc[4];
    for (int c = 0; c < 4; ++c) acc[c] = d4{0.0, 0.0, 0.0, (double)c};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  }
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

static float time_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  hipEventElapsedTime(&ms, a, b);
  return ms;
}

// LDS access cost probe: one wave issues `iters` x 8 LDS instructions of one
// kind, every lane at its own byte offset (< 8 KB, aligned to the access
// width) plus 8 KB x u for the u-th instruction of a group (the bank pattern
// repeats every 256 bytes, so all eight see the same banks).  Writes the
// elapsed shader clock cycles to *cycles.
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ __launch_bounds__(64) void k_lds_probe(const int* offs, int iters, long long* cycles,
                                                  int* sink) {
  __shared__ __align__(16) int lds[16384];   // 64 KB
  for (int i = threadIdx.x; i < 16384; i += 64) lds[i] = i;
  __syncthreads();
  const unsigned addr = (unsigned)(size_t)(__attribute__((address_space(3))) int*)lds + offs[threadIdx.x];
  v4i acc4 = {0, 0, 0, 0};
  v2i acc2 = {0, 0};
  const v4i w4 = {1, 2, 3, 4};
  const v2i w2 = {1, 2};
  __builtin_amdgcn_s_waitcnt(0);
  const long long t0 = __builtin_readcyclecounter();
  for (int it = 0; it < iters; ++it) {
    // the wait names the read results as operands, so nothing uses them
    // before the loads have landed
    if constexpr (KIND == 0) {
      v2i r0, r1, r2, r3, r4, r5, r6, r7;
#define RD(R, U) asm volatile("ds_read_b64 %0, %1 offset:%2" : "=v"(R) : "v"(addr), "i"(U * 8192));
      RD(r0, 0) RD(r1, 1) RD(r2, 2) RD(r3, 3) RD(r4, 4) RD(r5, 5) RD(r6, 6) RD(r7, 7)
#undef RD
      asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(r0), "+v"(r1), "+v"(r2), "+v"(r3), "+v"(r4),
                   "+v"(r5), "+v"(r6), "+v"(r7) : : "memory");
      acc2 ^= r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7;
    } else if constexpr (KIND == 1) {
      v4i r0, r1, r2, r3, r4, r5, r6, r7;
#define RD(R, U) asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(R) : "v"(addr), "i"(U * 8192));
      RD(r0, 0) RD(r1, 1) RD(r2, 2) RD(r3, 3) RD(r4, 4) RD(r5, 5) RD(r6, 6) RD(r7, 7)
#undef RD
      asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(r0), "+v"(r1), "+v"(r2), "+v"(r3), "+v"(r4),
                   "+v"(r5), "+v"(r6), "+v"(r7) : : "memory");
      acc4 ^= r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7;
    } else {
#define WR(U)                                                                              \
      if constexpr (KIND == 2)                                                             \
        asm volatile("ds_write_b64 %0, %1 offset:%2" : : "v"(addr), "v"(w2), "i"(U * 8192)); \
      else                                                                                 \
        asm volatile("ds_write_b128 %0, %1 offset:%2" : : "v"(addr), "v"(w4), "i"(U * 8192));
      WR(0) WR(1) WR(2) WR(3) WR(4) WR(5) WR(6) WR(7)
#undef WR
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
  }
  const long long t1 = __builtin_readcyclecounter();
  if (threadIdx.x == 0) *cycles = t1 - t0;
  sink[threadIdx.x] = acc4.x + acc4.y + acc4.z + acc4.w + acc2.x + acc2.y;
}

extern "C" {

// kind: 0 ds_read_b64, 1 ds_read_b128, 2 ds_write_b64, 3 ds_write_b128.
// offs: 64 device ints, each in [0, 8192 - width] and a multiple of the
// width (checked by the caller).  Returns 0 on success.
int mb_lds_probe(int kind, const int* offs, int iters, long long* cycles, int* sink) {
  switch (kind) {
    case 0: hipLaunchKernelGGL(k_lds_probe<0>, dim3(1), dim3(64), 0, 0, offs, iters, cycles, sink); break;
    case 1: hipLaunchKernelGGL(k_lds_probe<1>, dim3(1), dim3(64), 0, 0, offs, iters, cycles, sink); break;
    case 2: hipLaunchKernelGGL(k_lds_probe<2>, dim3(1), dim3(64), 0, 0, offs, iters, cycles, sink); break;
    default: hipLaunchKernelGGL(k_lds_probe<3>, dim3(1), dim3(64), 0, 0, offs, iters, cycles, sink); break;
  }
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

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

// mode selects (CBSZ, ABID): 0 (0,0), 1 (1,0), 2 (1,1), 3 (2,0), 4 (2,1),
// 5 (2,3), 6 (3,0).
int mb_mfma_f64_4x4x4(const double* a, const double* b, const double* c, double* d, int mode) {
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_mfma4_once<0, 0>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    case 1: hipLaunchKernelGGL((k_mfma4_once<1, 0>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    case 2: hipLaunchKernelGGL((k_mfma4_once<1, 1>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    case 3: hipLaunchKernelGGL((k_mfma4_once<2, 0>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    case 4: hipLaunchKernelGGL((k_mfma4_once<2, 1>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    case 5: hipLaunchKernelGGL((k_mfma4_once<2, 3>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
    default: hipLaunchKernelGGL((k_mfma4_once<3, 0>), dim3(1), dim3(64), 0, 0, a, b, c, d); break;
  }
  return hipDeviceSynchronize() == hipSuccess ? 0 : 1;
}

// kind: 0 = MFMA f64 (4 chains), 1 = vector FMA f64, 2 = mixed halves,
//       3 = MFMA f64 with 8 chains, 4 = 4x4x4 MFMA f64 with 8 chains.
// Returns the elapsed milliseconds of `reps` launches (negative on error).
double mb_fp64_peak_ms(int kind, int grid, int iters, int reps, double* sink) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&]() {
    if (kind == 0) hipLaunchKernelGGL(k_mfma_peak<4>, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
    else if (kind == 1) hipLaunchKernelGGL(k_valu_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
    else if (kind == 2) hipLaunchKernelGGL(k_mixed_peak, dim3(grid), dim3(256), 0, 0, sink, iters, 0.5);
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

// kind: 0 = copy (src -> dst, `bytes` each), 1 = read-only.
double mb_stream_ms(int kind, const void* src, void* dst, long long bytes, int grid, int reps,
                    double* sink) {
  const int64_t quad = 4ll * grid * 256;
  const int64_t n2 = (bytes / 16) / quad * quad;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  auto launch = [&]() {
    if (kind == 0)
      hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, (const double2*)src, (double2*)dst, n2);
    else
      hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, 0, (const double2*)src, n2, sink);
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
