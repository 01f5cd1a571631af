// Complex batched GEMM (the paper's matrices are complex, Section II, Eq. 1):
// C_i <- alpha op(A_i) op(B_i) + beta C_i with interleaved binary64 (real,
// imaginary) elements, op = N, T or C (conjugate transpose).
//
// The complex product is computed as the real product of embedded operands:
// with a = op(A)(r, p) and b = op(B)(p, c),
//     [Re C]   [Re a  -Im a] [Re b]
//     [Im C] = [Im a   Re a] [Im b]
// so op(A) becomes a real (2m x 2k) matrix A'' of 2 x 2 blocks and op(B) a
// real (2k x n) matrix B'' whose rows alternate real and imaginary parts.  The
// expansion happens while a tile is written to LDS; the contraction is then a
// real GEMM on the FP64 matrix cores, the same number of multiply-adds as four
// real products.
//
// LDS holds, per step, two planes of the embedded A (the real-part rows
// [Re a, -Im a] and the imaginary-part rows [Im a, Re a] over pairs of real
// k) and B's embedded rows [Re b; Im b], all k-major.  One
// v_mfma_f64_4x4x4_4b_f64 takes a 16-row slab of one plane (lane 16 s + r
// holds row r at real k s) and four B columns replicated over the four blocks
// (lane 16 s + 4 b + j holds column j), and yields a 16 x 4 block of the real
// or of the imaginary parts of C (lane 16 i + 4 b + j holds row 4 b + i,
// column j).  The two planes go to two accumulators, so the real and the
// imaginary part of each C element sit in one lane for the complex epilogue.
//
// Tile: 64 x 64 complex C per workgroup, four waves of 32 x 32, eight complex
// k per step (sixteen real k), double-buffered LDS, loads staged through
// registers one step ahead.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bgemm_internal.h"

namespace bg {
namespace cplx {

#define AS_GLOBAL __attribute__((address_space(1)))
#define AS_LDS __attribute__((address_space(3)))

constexpr int BM = 64, BN = 64, BK = 8, NT = 256;
constexpr int K2 = 2 * BK;          // real k of a step
// LDS row strides (doubles) of the A planes and of B's rows: the small pad keeps
// a stage at 26 KB, so three workgroups fit a CU (measured 52.0 vs 43.5
// TFLOP/s with a 16-double pad at two per CU)
#ifndef BG_ZPAD
#define BG_ZPAD 4
#endif
constexpr int SP = BM + BG_ZPAD;
constexpr int SB = BN + BG_ZPAD;
constexpr int PLANE = K2 * SP;
constexpr int STAGE = 2 * PLANE + K2 * SB;
constexpr int PER = BM * BK / NT;   // complex elements per thread per operand tile

struct Z {
  double re, im;
};

template <int TA, int TB>
struct Loader {
  Z a[PER], b[PER];

  // op codes: 0 N, 1 T, 2 C
  __device__ __forceinline__ void load(const AS_GLOBAL double* A, int64_t lda,
                                       const AS_GLOBAL double* B, int64_t ldb, int M, int N,
                                       int K, int m0, int n0, int k0, int tid) {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = tid + it * NT;
      // A tile element (row w, k q): coalesced along the contiguous index
      const int w = TA == 0 ? e % BM : e / BK;
      const int q = TA == 0 ? e / BM : e % BK;
      const int r = m0 + w, p = k0 + q;
      Z x{0.0, 0.0};
      if (r < M && p < K) {
        const AS_GLOBAL double* s = TA == 0 ? A + 2 * ((int64_t)r + (int64_t)p * lda)
                                            : A + 2 * ((int64_t)p + (int64_t)r * lda);
        x.re = s[0];
        x.im = TA == 2 ? -s[1] : s[1];
      }
      a[it] = x;
      // B tile element (k q, column c)
      const int q2 = TB == 0 ? e % BK : e / BN;
      const int c2 = TB == 0 ? e / BK : e % BN;
      const int p2 = k0 + q2, c = n0 + c2;
      Z y{0.0, 0.0};
      if (p2 < K && c < N) {
        const AS_GLOBAL double* s = TB == 0 ? B + 2 * ((int64_t)p2 + (int64_t)c * ldb)
                                            : B + 2 * ((int64_t)c + (int64_t)p2 * ldb);
        y.re = s[0];
        y.im = TB == 2 ? -s[1] : s[1];
      }
      b[it] = y;
    }
  }

  __device__ __forceinline__ void store(AS_LDS double* st, int tid) const {
    AS_LDS double* pre = st;              // rows [Re a, -Im a]
    AS_LDS double* pim = st + PLANE;      // rows [Im a,  Re a]
    AS_LDS double* lb = st + 2 * PLANE;
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = tid + it * NT;
      const int w = TA == 0 ? e % BM : e / BK;
      const int q = TA == 0 ? e / BM : e % BK;
      pre[(2 * q) * SP + w] = a[it].re;
      pre[(2 * q + 1) * SP + w] = -a[it].im;
      pim[(2 * q) * SP + w] = a[it].im;
      pim[(2 * q + 1) * SP + w] = a[it].re;
      const int q2 = TB == 0 ? e % BK : e / BN;
      const int c2 = TB == 0 ? e / BK : e % BN;
      lb[(2 * q2) * SB + c2] = b[it].re;
      lb[(2 * q2 + 1) * SB + c2] = b[it].im;
    }
  }
};

template <int TA, int TB>
__global__ __launch_bounds__(NT) void k_zgemm(int M, int N, int K, double ar, double ai,
                                              const double* const* __restrict__ Ap, int64_t lda,
                                              const double* const* __restrict__ Bp, int64_t ldb,
                                              double br, double bi, double* const* __restrict__ Cp,
                                              int64_t ldc, int tiles_m, int tiles_per_inst,
                                              int64_t total_tiles, int64_t per_xcd) {
  // the epilogue's complex products round as written (no fused multiply-add)
#pragma clang fp contract(off)
  __shared__ double lds_raw[2 * STAGE];
  AS_LDS double* lds = (AS_LDS double*)lds_raw;
  const int64_t bid = blockIdx.x;
  const int64_t id = (bid % 8) * per_xcd + bid / 8;   // contiguous tiles per XCD
  if (id >= total_tiles) return;
  const int64_t inst = id / tiles_per_inst;
  const int t = (int)(id - inst * tiles_per_inst);
  const int m0 = (t % tiles_m) * BM, n0 = (t / tiles_m) * BN;
  const AS_GLOBAL double* A = (const AS_GLOBAL double*)Ap[inst];
  const AS_GLOBAL double* B = (const AS_GLOBAL double*)Bp[inst];
  AS_GLOBAL double* C = (AS_GLOBAL double*)Cp[inst];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32;        // wave's first complex row
  const int wc = (wave >> 1) * 32;       // wave's first column
  const int ls = lane >> 4;              // real k within an instruction
  const int lr = lane & 15, lj = lane & 3;

  // acc[t][part][g]: slab t (16 rows), part (0 Re, 1 Im), column group g (4)
  double acc[2][2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int pt = 0; pt < 2; ++pt)
#pragma unroll
      for (int g = 0; g < 8; ++g) acc[t][pt][g] = 0.0;

  Loader<TA, TB> ld;
  const int nk = (K + BK - 1) / BK;
  ld.load(A, lda, B, ldb, M, N, K, m0, n0, 0, tid);
  ld.store(lds, tid);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) ld.load(A, lda, B, ldb, M, N, K, m0, n0, (kt + 1) * BK, tid);
    const AS_LDS double* pl = lds + cur * STAGE;
    const AS_LDS double* lb = pl + 2 * PLANE;
#pragma unroll
    for (int kk = 0; kk < K2; kk += 4) {
      double fp[2][2], fq[8];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
          fp[t][pt] = pl[pt * PLANE + (kk + ls) * SP + wr + 16 * t + lr];
#pragma unroll
      for (int g = 0; g < 8; ++g) fq[g] = lb[(kk + ls) * SB + wc + 4 * g + lj];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int pt = 0; pt < 2; ++pt)
#pragma unroll
          for (int g = 0; g < 8; ++g)
            acc[t][pt][g] =
                __builtin_amdgcn_mfma_f64_4x4x4f64(fp[t][pt], fq[g], acc[t][pt][g], 0, 0, 0);
    }
    if (kt + 1 < nk) ld.store(lds + (cur ^ 1) * STAGE, tid);
    __syncthreads();
  }

  // Epilogue: lane 16 i + 4 b + j holds row wr + 16 t + 4 b + i, column
  // wc + 4 g + j of slab t, group g (real part in acc[t][0][g], imaginary in
  // acc[t][1][g]).
  const bool read_c = !(br == 0.0 && bi == 0.0);
  const int li = lane >> 4, lb4 = (lane >> 2) & 3;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int r = m0 + wr + 16 * t + 4 * lb4 + li;
      const int c = n0 + wc + 4 * g + lj;
      if (r >= M || c >= N) continue;
      const double sr = acc[t][0][g], si = acc[t][1][g];
      double xr = ar * sr - ai * si;
      double xi = ar * si + ai * sr;
      AS_GLOBAL double* dst = C + 2 * ((int64_t)r + (int64_t)c * ldc);
      if (read_c) {
        const double cr = dst[0], ci = dst[1];
        const double yr = br * cr - bi * ci;
        const double yi = br * ci + bi * cr;
        xr = xr + yr;
        xi = xi + yi;
      }
      dst[0] = xr;
      dst[1] = xi;
    }
}

// C <- beta C (complex), exactly zero when beta == 0 (C not read).
__global__ __launch_bounds__(256) void k_zscale(double br, double bi, double* const* __restrict__ Cp,
                                                int64_t ldc, int m, int n, int64_t total_cols) {
#pragma clang fp contract(off)
  for (int64_t col = blockIdx.x; col < total_cols; col += gridDim.x) {
    const int64_t inst = col / n;
    const int c = (int)(col - inst * n);
    double* base = Cp[inst] + 2 * (int64_t)c * ldc;
    for (int r = threadIdx.x; r < m; r += 256) {
      double* z = base + 2 * r;
      if (br == 0.0 && bi == 0.0) {
        z[0] = 0.0;
        z[1] = 0.0;
      } else {
        const double cr = z[0], ci = z[1];
        z[0] = br * cr - bi * ci;
        z[1] = br * ci + bi * cr;
      }
    }
  }
}

template <int TA, int TB>
static hipError_t launch(const ZUniformArgs& a, hipStream_t s) {
  const int tiles_m = (a.m + BM - 1) / BM, tiles_n = (a.n + BN - 1) / BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int64_t total = tpi * a.batch;
  const int64_t per_xcd = (total + 7) / 8;
  if (tpi > INT32_MAX || per_xcd * 8 > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_zgemm<TA, TB>), dim3((unsigned)(per_xcd * 8)), dim3(NT), 0, s, a.m, a.n,
                     a.k, a.alpha[0], a.alpha[1], a.A, a.lda, a.B, a.ldb, a.beta[0], a.beta[1],
                     a.C, a.ldc, tiles_m, (int)tpi, total, per_xcd);
  return hipGetLastError();
}

}  // namespace cplx

hipError_t launch_zgemm(const ZUniformArgs& a, hipStream_t s) {
  using namespace cplx;
  switch (a.ta * 3 + a.tb) {
    case 0: return launch<0, 0>(a, s);
    case 1: return launch<0, 1>(a, s);
    case 2: return launch<0, 2>(a, s);
    case 3: return launch<1, 0>(a, s);
    case 4: return launch<1, 1>(a, s);
    case 5: return launch<1, 2>(a, s);
    case 6: return launch<2, 0>(a, s);
    case 7: return launch<2, 1>(a, s);
    default: return launch<2, 2>(a, s);
  }
}

hipError_t launch_zscale(const double* beta, double* const* C, int64_t ldc, int m, int n,
                         int batch, hipStream_t s) {
  const int64_t cols = (int64_t)n * batch;
  if (cols <= 0) return hipSuccess;
  const int64_t grid = cols < 65536 ? cols : 65536;
  hipLaunchKernelGGL(cplx::k_zscale, dim3((unsigned)grid), dim3(256), 0, s, beta[0], beta[1], C,
                     ldc, m, n, cols);
  return hipGetLastError();
}

}  // namespace bg
