// Reduced- and emulated-precision batched GEMM modes for gfx950.
//
// Same operation as the FP64 path (the paper, Section II, Eq. 1), on binary64
// inputs and outputs, with cheaper inner arithmetic:
//   fp32 : inputs rounded to binary32, products and sums on the binary32
//          matrix cores (v_mfma_f32_16x16x4_f32);
//   bf16 : inputs rounded to binary32 then bfloat16 (nearest even), binary32
//          accumulation (v_mfma_f32_16x16x32_bf16);
//   emu  : emulated binary64 from S bfloat16 digit slices.  Per 32-wide chunk
//          of k, row i of A and column j of B are scaled by powers of two
//          2^-e_i, 2^-f_j (frexp exponent of the chunk's largest magnitude)
//          into (-1, 1); each value is split into digits d_1 = rint(x 2^7),
//          d_t = rint(r_{t-1} 2^8) with remainders r_t (integers in
//          [-128, 128], exact in bfloat16); for each diagonal g = t + u <=
//          S + 1 the integer sums S_g = sum dA_t dB_u are accumulated on the
//          bfloat16 matrix cores in binary32 (exact: |S_g| < 2^24); then in
//          binary64: T = sum over g from S+1 down to 2 of S_g 2^(-14-8(g-2)),
//          V = T 2^(e_i + f_j), acc += V over chunks in ascending order.
//          Every rounding is fixed in kind and order, so the result is
//          reproducible bit for bit by a CPU implementation of these steps.
//   emu32: the same digits and sums on the binary32 matrix cores
//          (v_mfma_f32_16x16x4_f32, digits converted exactly to binary32):
//          every digit product and every partial sum is an integer below
//          2^24, so the sums, and the whole result, are bit-identical to emu.
//
// Tile: 64 x 64 of C per workgroup (four waves of 32 x 32, i.e. 2 x 2 blocks
// of 16 x 16), one 32-wide chunk of k per step.  Each step stages the binary64
// tiles in LDS, converts them to the mode's operand tiles in LDS (k
// contiguous per row of A / column of B), then runs the matrix-core
// instructions.  The instruction's first operand is B's tile and its second
// A's, so a result block is the transpose of a C block and its 16 lanes cover
// 16 consecutive rows of a C column (coalesced epilogue).  Operands must be
// non-transposed (NN).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bgemm_internal.h"

namespace bg {
namespace lowp {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

#define AS_GLOBAL __attribute__((address_space(1)))
#define AS_LDS __attribute__((address_space(3)))

constexpr int BM = 64, BN = 64, BKC = 32, NT = 256;
constexpr int S64A = BM + 2;    // staging A: [k][m], doubles
constexpr int S64B = BKC + 1;   // staging B: [n][k], doubles
constexpr int SF = BKC + 4;     // fp32 operand rows (floats): bank-distinct 4-byte reads
constexpr int SH = BKC + 8;     // bf16 operand rows (halves): 80-byte stride, distinct 16-byte reads

enum Mode { FP32 = 1, BF16 = 2, EMU = 3, EMU32 = 5 };

// a digit held as bfloat16 bits, as the binary32 value it represents (exact)
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float((unsigned int)h << 16);
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// a value that bfloat16 holds exactly (a digit): its top 16 bits
__device__ __forceinline__ unsigned short bf16_exact(float f) {
  return (unsigned short)(__float_as_uint(f) >> 16);
}

// the digit-slice modes
constexpr bool is_emu(int mode) { return mode == EMU || mode == EMU32; }

template <int MODE, int S>
struct __align__(16) Smem {
  static constexpr int NSL = is_emu(MODE) ? S : 1;
  double a64[BKC * S64A];
  double b64[BN * S64B];
  int ea[BM], fb[BN];
  union {
    struct { float a[BM * SF]; float b[BN * SF]; } f32;
    struct { unsigned short a[NSL][BM * SH]; unsigned short b[NSL][BN * SH]; } h16;
  } op;
};

template <int MODE, int S>
__global__ __launch_bounds__(NT) void k_lowp(int M, int N, int K, double alpha,
                                             const double* const* __restrict__ Ap, int64_t lda,
                                             const double* const* __restrict__ Bp, int64_t ldb,
                                             double beta, double* const* __restrict__ Cp,
                                             int64_t ldc, int tiles_m, int tiles_per_inst,
                                             int64_t total_tiles, int64_t per_xcd) {
  // every binary64 rounding below is the one written (no fused multiply-add),
  // which is what makes the emulated mode reproducible bit for bit
#pragma clang fp contract(off)
  __shared__ Smem<MODE, S> sm;
  constexpr int NG = is_emu(MODE) ? S : 1;   // accumulator sets (diagonals g = 2..S+1)
  const int64_t bid = blockIdx.x;
  const int64_t id = (bid % 8) * per_xcd + bid / 8;   // contiguous tiles per XCD
  if (id >= total_tiles) return;
  const int64_t inst = id / tiles_per_inst;
  const int tt = (int)(id - inst * tiles_per_inst);
  const int m0 = (tt % tiles_m) * BM, n0 = (tt / tiles_m) * BN;
  const AS_GLOBAL double* A = (const AS_GLOBAL double*)Ap[inst];
  const AS_GLOBAL double* B = (const AS_GLOBAL double*)Bp[inst];
  AS_GLOBAL double* C = (AS_GLOBAL double*)Cp[inst];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;
  const int li = lane & 15, lg = lane >> 4;

  f4 acc32[NG][2][2];
  double acc64[2][2][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc32[g][bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[bi][bj][v] = 0.0;

  const bool use_product = !(alpha == 0.0 || K == 0);
  const int nchunks = use_product ? (K + BKC - 1) / BKC : 0;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int k0 = ch * BKC;
    // 1. stage the binary64 tiles (zero outside the matrix)
#pragma unroll
    for (int it = 0; it < (BM * BKC) / NT; ++it) {   // A: 32 columns of 64 rows
      const int e = tid + it * NT, r = e % BM, kk = e / BM;
      const int gr = m0 + r, gk = k0 + kk;
      sm.a64[kk * S64A + r] = (gr < M && gk < K) ? A[gr + (int64_t)gk * lda] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < (BN * BKC) / NT; ++it) {   // B: 64 columns of 32 k
      const int e = tid + it * NT, kk = e % BKC, c = e / BKC;
      const int gc = n0 + c, gk = k0 + kk;
      sm.b64[c * S64B + kk] = (gc < N && gk < K) ? B[gk + (int64_t)gc * ldb] : 0.0;
    }
    __syncthreads();
    // 2. (emu) chunk exponents of the 64 rows of A and 64 columns of B
    if constexpr (is_emu(MODE)) {
      if (tid < BM) {
        double mx = 0.0;
        for (int kk = 0; kk < BKC; ++kk) mx = fmax(mx, fabs(sm.a64[kk * S64A + tid]));
        int e = 0;
        if (mx > 0.0) frexp(mx, &e);
        sm.ea[tid] = e;
      } else if (tid < BM + BN) {
        const int c = tid - BM;
        double mx = 0.0;
        for (int kk = 0; kk < BKC; ++kk) mx = fmax(mx, fabs(sm.b64[c * S64B + kk]));
        int e = 0;
        if (mx > 0.0) frexp(mx, &e);
        sm.fb[c] = e;
      }
      __syncthreads();
    }
    // 3. operand tiles: thread handles 8 consecutive k of one row of A and of
    //    one column of B (row / column = tid % 64, k block = tid / 64)
    {
      const int r = tid % 64, kb = (tid / 64) * 8;
      double xa[8], xb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        xa[e] = sm.a64[(kb + e) * S64A + r];
        xb[e] = sm.b64[r * S64B + kb + e];
      }
      if constexpr (MODE == FP32) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          sm.op.f32.a[r * SF + kb + e] = (float)xa[e];
          sm.op.f32.b[r * SF + kb + e] = (float)xb[e];
        }
      } else if constexpr (MODE == BF16) {
        u16x8 ha, hb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ha[e] = bf16_rne((float)xa[e]);
          hb[e] = bf16_rne((float)xb[e]);
        }
        *(u16x8*)&sm.op.h16.a[0][r * SH + kb] = ha;
        *(u16x8*)&sm.op.h16.b[0][r * SH + kb] = hb;
      } else {
        const int ea = sm.ea[r], fb = sm.fb[r];
        double ra[8], rb[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          ra[e] = ldexp(xa[e], -ea) * 128.0;
          rb[e] = ldexp(xb[e], -fb) * 128.0;
        }
#pragma unroll
        for (int t = 0; t < S; ++t) {
          u16x8 ha, hb;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const double da = rint(ra[e]), db = rint(rb[e]);
            ha[e] = bf16_exact((float)da);
            hb[e] = bf16_exact((float)db);
            ra[e] = (ra[e] - da) * 256.0;
            rb[e] = (rb[e] - db) * 256.0;
          }
          *(u16x8*)&sm.op.h16.a[t][r * SH + kb] = ha;
          *(u16x8*)&sm.op.h16.b[t][r * SH + kb] = hb;
        }
      }
    }
    __syncthreads();
    // 4. matrix-core products
    if constexpr (MODE == FP32) {
#pragma unroll
      for (int ks = 0; ks < BKC; ks += 4) {
        float fa[2], fbv[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          fa[b] = sm.op.f32.a[(wm0 + 16 * b + li) * SF + ks + lg];
          fbv[b] = sm.op.f32.b[(wn0 + 16 * b + li) * SF + ks + lg];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc32[0][bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(fbv[bj], fa[bi], acc32[0][bi][bj], 0, 0, 0);
      }
    } else if constexpr (MODE == EMU32) {
      // per diagonal pair (t, u): eight 4-wide steps of k on the binary32
      // matrix cores; lane (li, lg) takes digit k = ks + lg of row / column li
#pragma unroll
      for (int t = 1; t <= S; ++t) {
#pragma unroll
        for (int u = 1; u <= S; ++u) {
          if (t + u > S + 1) continue;
          const int g = t + u - 2;
#pragma unroll
          for (int ks = 0; ks < BKC; ks += 4) {
            float fa[2], fbv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              fa[b] = bf16_to_f32(sm.op.h16.a[t - 1][(wm0 + 16 * b + li) * SH + ks + lg]);
              fbv[b] = bf16_to_f32(sm.op.h16.b[u - 1][(wn0 + 16 * b + li) * SH + ks + lg]);
            }
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
              for (int bj = 0; bj < 2; ++bj)
                acc32[g][bi][bj] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(fbv[bj], fa[bi], acc32[g][bi][bj], 0, 0, 0);
          }
        }
      }
    } else {
#pragma unroll
      for (int t = 1; t <= (MODE == EMU ? S : 1); ++t) {
        bf8 va[2];
#pragma unroll
        for (int b = 0; b < 2; ++b)
          va[b] = __builtin_bit_cast(bf8, *(const u16x8*)&sm.op.h16.a[t - 1][(wm0 + 16 * b + li) * SH + 8 * lg]);
#pragma unroll
        for (int u = 1; u <= (MODE == EMU ? S : 1); ++u) {
          if (t + u > S + 1 && MODE == EMU) continue;
          bf8 vb[2];
#pragma unroll
          for (int b = 0; b < 2; ++b)
            vb[b] = __builtin_bit_cast(bf8, *(const u16x8*)&sm.op.h16.b[u - 1][(wn0 + 16 * b + li) * SH + 8 * lg]);
          const int g = MODE == EMU ? t + u - 2 : 0;
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
              acc32[g][bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vb[bj], va[bi], acc32[g][bi][bj], 0, 0, 0);
        }
      }
    }
    if constexpr (MODE != FP32) {
      // 5. (emu) fold this chunk into binary64 in the fixed order
      if constexpr (is_emu(MODE)) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              // lane holds C(row = wm0 + 16 bi + li, col = wn0 + 16 bj + 4 lg + v)
              double T = 0.0;
#pragma unroll
              for (int g = S - 1; g >= 0; --g)   // diagonal t + u = g + 2, largest first
                T = T + (double)acc32[g][bi][bj][v] * ldexp(1.0, -14 - 8 * g);
              const int er = sm.ea[wm0 + 16 * bi + li], fc = sm.fb[wn0 + 16 * bj + 4 * lg + v];
              acc64[bi][bj][v] = acc64[bi][bj][v] + ldexp(T, er + fc);
            }
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
          for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc32[g][bi][bj] = f4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();   // before the next chunk overwrites the LDS tiles
  }

  // epilogue: lane holds C(m0 + wm0 + 16 bi + li, n0 + wn0 + 16 bj + 4 lg + v)
  double cv[2][2][4];
  if (beta != 0.0) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm0 + 16 * bi + li, col = n0 + wn0 + 16 * bj + 4 * lg + v;
          cv[bi][bj][v] = (row < M && col < N) ? C[row + (int64_t)col * ldc] : 0.0;
        }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + 16 * bi + li, col = n0 + wn0 + 16 * bj + 4 * lg + v;
        if (row >= M || col >= N) continue;
        double x;
        if (!use_product) {
          if (beta == 1.0) continue;
          x = beta == 0.0 ? 0.0 : beta * cv[bi][bj][v];
        } else {
          const double p = is_emu(MODE) ? acc64[bi][bj][v] : (double)acc32[0][bi][bj][v];
          x = alpha * p;
          if (beta != 0.0) x = x + beta * cv[bi][bj][v];
        }
        C[row + (int64_t)col * ldc] = x;
      }
}

template <int MODE, int S>
static hipError_t launch(const UniformArgs& a, hipStream_t s) {
  const int tiles_m = (a.m + BM - 1) / BM, tiles_n = (a.n + BN - 1) / BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int64_t total = tpi * a.batch;
  const int64_t per_xcd = (total + 7) / 8;
  if (tpi > INT32_MAX || per_xcd * 8 > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_lowp<MODE, S>), dim3((unsigned)(per_xcd * 8)), dim3(NT), 0, s, a.m, a.n, a.k,
                     a.alpha, a.A, a.lda, a.B, a.ldb, a.beta, a.C, a.ldc, tiles_m, (int)tpi, total,
                     per_xcd);
  return hipGetLastError();
}

}  // namespace lowp

hipError_t launch_uniform_lowp(const UniformArgs& a, int mode, int slices, hipStream_t s) {
  using namespace lowp;
  if (mode == FP32) return launch<FP32, 1>(a, s);
  if (mode == BF16) return launch<BF16, 1>(a, s);
  if (mode == EMU32) {
    switch (slices) {
      case 1: return launch<EMU32, 1>(a, s);
      case 2: return launch<EMU32, 2>(a, s);
      case 3: return launch<EMU32, 3>(a, s);
      case 4: return launch<EMU32, 4>(a, s);
      case 5: return launch<EMU32, 5>(a, s);
      case 6: return launch<EMU32, 6>(a, s);
      case 7: return launch<EMU32, 7>(a, s);
      case 8: return launch<EMU32, 8>(a, s);
    }
    return hipErrorInvalidValue;
  }
  switch (slices) {
    case 1: return launch<EMU, 1>(a, s);
    case 2: return launch<EMU, 2>(a, s);
    case 3: return launch<EMU, 3>(a, s);
    case 4: return launch<EMU, 4>(a, s);
    case 5: return launch<EMU, 5>(a, s);
    case 6: return launch<EMU, 6>(a, s);
    case 7: return launch<EMU, 7>(a, s);
    case 8: return launch<EMU, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bg
