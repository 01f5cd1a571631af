// Emulated binary64 batched GEMM on the int8 matrix cores of gfx950
// (v_mfma_i32_16x16x64_i8), the i8emu<S> mode.
//
// Same operation as the FP64 path (the paper, Section II, Eq. 1), on binary64
// inputs and outputs.  The error-free splitting follows Ozaki, Ogita, Oishi
// and Rump (Numer. Algorithms 59, 2012), with integer digits:
//   1. e_i: frexp exponent of the largest |A(i, p)| over the whole row i of A;
//      f_j likewise for column j of B (kernel k_exp, one pass over A and B).
//   2. X = rint(A(i, p) 2^(8S-2-e_i)), an integer with |X| <= 2^(8S-2);
//      Y likewise for B.
//   3. Signed base-256 digits X = sum_t d_t 256^(S-t), d_t in [-128, 127]
//      (d_1 in [-64, 64]): with Z = X + 0x80..80 (S bytes), digit d_t is byte
//      S-t of Z minus 128, i.e. that byte with its top bit flipped, read as
//      an int8.
//   4. For each diagonal g = t + u <= S + 1, S_g = sum_p sum_{t+u=g}
//      dA_t(i, p) dB_u(p, j) on the int8 matrix cores in int32: exact, since
//      |S_g| <= S k 2^14 < 2^31 for k <= 8192.  Exact integers do not depend on
//      the order of the sum, so any blocking of k gives the same S_g.
//   5. In binary64: T = S_{S+1}; T = S_g + T 2^-8 for g = S .. 2;
//      V = T 2^(e_i + f_j - 12); C = alpha V (+ beta C).
// Every rounding is fixed in kind and order, so the result equals a CPU
// implementation of these steps bit for bit.
//
// Main kernel: one 128 x 64 C tile per workgroup of eight waves (each 32 x 32,
// 2 x 2 blocks of 16 x 16), 64 of k per step.  Each thread loads 16 binary64
// values of A (one row, 16 consecutive k) and 8 of B (one column, 8
// consecutive k), turns them into S digit bytes each and writes one word per
// digit plane to LDS (rows of 64 digits, 80-byte stride); then each wave runs
// S (S + 1) / 2 x 4 int8 matrix-core instructions into S int32 accumulator
// sets.  The instruction's first operand is B's digits and its second A's, so
// a result block is the transpose of a C block and its 16 lanes cover 16
// consecutive rows of a C column (coalesced epilogue).  NN operands only.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bgemm_internal.h"

namespace bg {
namespace emu8 {

typedef int i4 __attribute__((ext_vector_type(4)));
#define AS_GLOBAL __attribute__((address_space(1)))
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef double d2 __attribute__((ext_vector_type(2)));

#ifndef BG_EMU8_BM
#define BG_EMU8_BM 128
#endif
// C tile: TM x 64 (TM = 64: four waves; 128: eight waves), 64 of k per step
constexpr int TM = BG_EMU8_BM, BN = 64, BK = 64, NT = TM * 4;
static_assert(TM == 64 || TM == 128, "tile height");
constexpr int RS = BK + 16;            // bytes per digit row in LDS
constexpr int PLANE_A = TM * RS;       // bytes per digit plane of A (TM rows)
constexpr int PLANE_B = 64 * RS;       // bytes per digit plane of B (64 columns)
constexpr int EXP_COLS = 16;           // columns of B per exponent block

// ---- exponents ------------------------------------------------------------

__device__ __forceinline__ int frexp_exp(double mx) {
  int e = 0;
  (void)frexp(mx, &e);
  return mx > 0.0 ? e : 0;
}

// Blocks [0, nb_a) of an instance: one row of A per thread; blocks
// [nb_a, nb_a + nb_b): EXP_COLS columns of B, one wave per column at a time.
__global__ __launch_bounds__(256) void k_exp(int M, int N, int K,
                                             const double* const* __restrict__ Ap, int64_t lda,
                                             const double* const* __restrict__ Bp, int64_t ldb,
                                             int* __restrict__ ea, int* __restrict__ fb, int nb_a,
                                             int per_inst) {
  const int64_t inst = blockIdx.x / per_inst;
  const int blk = (int)(blockIdx.x - inst * per_inst);
  if (blk < nb_a) {
    const int r = blk * 256 + threadIdx.x;
    if (r >= M) return;
    const double* A = Ap[inst] + r;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
    int p = 0;
    for (; p + 4 <= K; p += 4) {
      m0 = fmax(m0, fabs(A[(int64_t)p * lda]));
      m1 = fmax(m1, fabs(A[(int64_t)(p + 1) * lda]));
      m2 = fmax(m2, fabs(A[(int64_t)(p + 2) * lda]));
      m3 = fmax(m3, fabs(A[(int64_t)(p + 3) * lda]));
    }
    for (; p < K; ++p) m0 = fmax(m0, fabs(A[(int64_t)p * lda]));
    ea[inst * M + r] = frexp_exp(fmax(fmax(m0, m1), fmax(m2, m3)));
  } else {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = (blk - nb_a) * EXP_COLS;
    for (int c = c0 + wave; c < c0 + EXP_COLS && c < N; c += 4) {
      const double* B = Bp[inst] + (int64_t)c * ldb;
      double mx = 0.0;
      for (int p = lane; p < K; p += 64) mx = fmax(mx, fabs(B[p]));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
      if (lane == 0) fb[inst * N + c] = frexp_exp(mx);
    }
  }
}

// ---- digits ---------------------------------------------------------------

// Z = X + 0x80..80 (S bytes) for x = rint(v 2^sh): low and high words.
template <int S>
__device__ __forceinline__ void z_words(double v, int sh, unsigned& lo, unsigned& hi) {
  const double x = rint(ldexp(v, sh));
  if constexpr (S <= 4) {
    constexpr unsigned ML = (unsigned)(0x80808080ull >> (8 * (4 - S)));
    lo = (unsigned)(int)x + ML;
    hi = 0;
  } else {
    constexpr unsigned MH = (unsigned)(0x80808080ull >> (8 * (8 - S)));
    const double h = floor(x * 0x1p-32);      // exact: |x| <= 2^62
    const double l = x - h * 0x1p32;           // exact, in [0, 2^32)
    const uint64_t z = (((uint64_t)(unsigned)(int)h << 32) | (uint64_t)(unsigned)l) +
                       (((uint64_t)MH << 32) | 0x80808080ull);
    lo = (unsigned)z;
    hi = (unsigned)(z >> 32);
  }
}

// 4 x 4 byte transpose: out[b] = [w0.b, w1.b, w2.b, w3.b] (first word in the
// low byte), for the NB lowest bytes b.  v_perm_b32 picks bytes of
// {src0 (high), src1 (low)}: selectors 0-3 address src1, 4-7 src0.
template <int NB>
__device__ __forceinline__ void transpose4(unsigned w0, unsigned w1, unsigned w2, unsigned w3,
                                           unsigned (&out)[4]) {
  const unsigned l01 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);   // w0.0 w1.0 w0.1 w1.1
  const unsigned l23 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);   // w2.0 w3.0 w2.1 w3.1
  out[0] = __builtin_amdgcn_perm(l23, l01, 0x05040100u);
  if constexpr (NB > 1) out[1] = __builtin_amdgcn_perm(l23, l01, 0x07060302u);
  if constexpr (NB > 2) {
    const unsigned h01 = __builtin_amdgcn_perm(w1, w0, 0x07030602u); // w0.2 w1.2 w0.3 w1.3
    const unsigned h23 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
    out[2] = __builtin_amdgcn_perm(h23, h01, 0x05040100u);
    if constexpr (NB > 3) out[3] = __builtin_amdgcn_perm(h23, h01, 0x07060302u);
  }
}

// NV values (consecutive k, NV = 8 or 16) -> S digit planes, one NV-byte word
// each, at dst + t * plane (t = 0 the most significant digit).
template <int S, int NV>
__device__ __forceinline__ void split(const double (&v)[NV], int sh, unsigned char* dst, int plane) {
  constexpr int NL = S < 4 ? S : 4, NH = S - NL, NQ = NV / 4;
  unsigned w[S][NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    unsigned lo[4], hi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) z_words<S>(v[4 * q + j], sh, lo[j], hi[j]);
    unsigned bl[4], bh[4];
    transpose4<NL>(lo[0], lo[1], lo[2], lo[3], bl);
#pragma unroll
    for (int b = 0; b < NL; ++b) w[S - 1 - b][q] = bl[b] ^ 0x80808080u;
    if constexpr (NH > 0) {
      transpose4<NH>(hi[0], hi[1], hi[2], hi[3], bh);
#pragma unroll
      for (int b = 0; b < NH; ++b) w[S - 5 - b][q] = bh[b] ^ 0x80808080u;
    }
  }
#pragma unroll
  for (int t = 0; t < S; ++t) {
    if constexpr (NQ == 4) *(u4*)(dst + t * plane) = u4{w[t][0], w[t][1], w[t][2], w[t][3]};
    else *(u2*)(dst + t * plane) = u2{w[t][0], w[t][1]};
  }
}

// ---- main kernel ----------------------------------------------------------

// x if ok, else +0.0, by masking its bits: the value is used either way, so
// the compiler keeps the load unconditional (no branch and wait per load)
__device__ __forceinline__ double keep(double x, bool ok) {
  const uint64_t m = ok ? ~0ull : 0ull;
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) & m);
}

template <int S>
__global__ __launch_bounds__(NT, 2) void k_emu8(int M, int N, int K, double alpha,
                                                const double* const* __restrict__ Ap, int64_t lda,
                                                const double* const* __restrict__ Bp, int64_t ldb,
                                                double beta, double* const* __restrict__ Cp,
                                                int64_t ldc, const int* __restrict__ ea,
                                                const int* __restrict__ fb, int tiles_m,
                                                int tiles_per_inst, int64_t total_tiles,
                                                int64_t per_xcd) {
  // every binary64 rounding below is the one written (no fused multiply-add)
#pragma clang fp contract(off)
  __shared__ __align__(16) unsigned char lds[S * (PLANE_A + PLANE_B)];
  unsigned char* la = lds;
  unsigned char* lb = lds + S * PLANE_A;
  const int64_t bid = blockIdx.x;
  const int64_t id = (bid % 8) * per_xcd + bid / 8;   // contiguous tiles per XCD
  if (id >= total_tiles) return;
  const int64_t inst = id / tiles_per_inst;
  const int tt = (int)(id - inst * tiles_per_inst);
  const int m0 = (tt % tiles_m) * TM, n0 = (tt / tiles_m) * BN;
  const AS_GLOBAL double* A = (const AS_GLOBAL double*)Ap[inst];
  const AS_GLOBAL double* B = (const AS_GLOBAL double*)Bp[inst];
  AS_GLOBAL double* C = (AS_GLOBAL double*)Cp[inst];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // split roles: A row m0 + ar, k = 16 akg .. +15; B column n0 + bc, k = BV bkq .. +BV-1
  constexpr int BV = 64 * 64 / NT;     // B values per thread: 16 (TM 64) or 8 (TM 128)
  const int ar = tid % TM, akg = tid / TM;
  const int bc = tid / (64 / BV), bkq = tid % (64 / BV);
  const bool a_ok = m0 + ar < M, b_ok = n0 + bc < N;
  // rows / columns outside the matrix get a shift that makes every value 0
  const int ash = a_ok ? (8 * S - 2) - ea[inst * M + m0 + ar] : -4096;
  const int bsh = b_ok ? (8 * S - 2) - fb[inst * N + n0 + bc] : -4096;
  // out-of-range rows / columns read a valid address (row / column 0);
  // every load of a step is issued before the first wait
  const AS_GLOBAL double* arow = A + (a_ok ? m0 + ar : 0);
  const AS_GLOBAL double* bcol = B + (int64_t)(b_ok ? n0 + bc : 0) * ldb;
  const bool b_vec = ((((uintptr_t)B) & 15) == 0) && ((ldb & 1) == 0);

  // wave tile: rows wm0 .. +31, columns wn0 .. +31 of the C tile
  const int wm0 = (wave % (TM / 32)) * 32, wn0 = (wave / (TM / 32)) * 32;
  const int li = lane & 15, lg = lane >> 4;

  i4 acc[S][2][2];
#pragma unroll
  for (int g = 0; g < S; ++g)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[g][bi][bj] = i4{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    double av[16], bv[BV];
    const int ka = k0 + 16 * akg, kb = k0 + BV * bkq;
    if (k0 + BK <= K) {
      // whole step inside k (uniform): plain loads; rows / columns outside
      // the matrix read row / column 0 and their shift of -4096 zeroes them
      const AS_GLOBAL double* pa = arow + (int64_t)ka * lda;
#pragma unroll
      for (int j = 0; j < 16; ++j) av[j] = pa[(int64_t)j * lda];
      if (b_vec) {
        const AS_GLOBAL d2* p = (const AS_GLOBAL d2*)(bcol + kb);
#pragma unroll
        for (int j = 0; j < BV / 2; ++j) {
          const d2 x = p[j];
          bv[2 * j] = x.x;
          bv[2 * j + 1] = x.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < BV; ++j) bv[j] = bcol[kb + j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        av[j] = keep(arow[(int64_t)min(ka + j, K - 1) * lda], ka + j < K);
#pragma unroll
      for (int j = 0; j < BV; ++j) bv[j] = keep(bcol[min(kb + j, K - 1)], kb + j < K);
    }
    __syncthreads();   // the previous step's digit reads are done
    split<S, 16>(av, ash, la + ar * RS + 16 * akg, PLANE_A);
    split<S, BV>(bv, bsh, lb + bc * RS + BV * bkq, PLANE_B);
    __syncthreads();

    i4 af[S][2];
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        af[t][bi] = *(const i4*)(la + t * PLANE_A + (wm0 + 16 * bi + li) * RS + 16 * lg);
#pragma unroll
    for (int u = 0; u < S; ++u) {
      i4 bf[2];
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        bf[bj] = *(const i4*)(lb + u * PLANE_B + (wn0 + 16 * bj + li) * RS + 16 * lg);
#pragma unroll
      for (int t = 0; t + u < S; ++t)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[t + u][bi][bj] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(bf[bj], af[t][bi], acc[t + u][bi][bj], 0, 0, 0);
    }
  }

  // epilogue: lane (li, lg), register v of block (bi, bj) holds the diagonal
  // sums of C(row m0 + wm0 + 16 bi + li, column n0 + wn0 + 16 bj + 4 lg + v)
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int row = m0 + wm0 + 16 * bi + li;
    if (row >= M) continue;
    const int er = ea[inst * M + row];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = n0 + wn0 + 16 * bj + 4 * lg + v;
        if (col >= N) continue;
        double T = (double)acc[S - 1][bi][bj][v];
#pragma unroll
        for (int g = S - 2; g >= 0; --g) T = (double)acc[g][bi][bj][v] + T * 0x1p-8;
        const double V = ldexp(T, er + fb[inst * N + col] - 12);
        AS_GLOBAL double* cp = C + row + (int64_t)col * ldc;
        double x = alpha * V;
        if (beta != 0.0) x = x + beta * *cp;
        *cp = x;
      }
  }
}

template <int S>
static hipError_t launch_group(const UniformArgs& a, int64_t b0, int g, int* ea, int* fb,
                               hipStream_t s) {
  const int nb_a = (a.m + 255) / 256, nb_b = (a.n + EXP_COLS - 1) / EXP_COLS;
  const int per_inst = nb_a + nb_b;
  hipLaunchKernelGGL(k_exp, dim3((unsigned)((int64_t)per_inst * g)), dim3(256), 0, s, a.m, a.n,
                     a.k, a.A + b0, a.lda, a.B + b0, a.ldb, ea, fb, nb_a, per_inst);
  const int tiles_m = (a.m + TM - 1) / TM, tiles_n = (a.n + BN - 1) / BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int64_t total = tpi * g;
  const int64_t per_xcd = (total + 7) / 8;
  hipLaunchKernelGGL((k_emu8<S>), dim3((unsigned)(per_xcd * 8)), dim3(NT), 0, s, a.m, a.n, a.k,
                     a.alpha, a.A + b0, a.lda, a.B + b0, a.ldb, a.beta, a.C + b0, a.ldc, ea, fb,
                     tiles_m, (int)tpi, total, per_xcd);
  return hipGetLastError();
}

template <int S>
static hipError_t launch(const UniformArgs& a, void* ws, size_t ws_bytes, hipStream_t s) {
  const int64_t per = (int64_t)(a.m + a.n) * (int64_t)sizeof(int);
  int64_t gmax = (int64_t)(ws_bytes / (size_t)per);
  const int tiles_m = (a.m + TM - 1) / TM, tiles_n = (a.n + BN - 1) / BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int nb = (a.m + 255) / 256 + (a.n + EXP_COLS - 1) / EXP_COLS;
  // grid sizes stay within 32 bits
  gmax = std::min<int64_t>(gmax, (int64_t)(INT32_MAX - 8) / std::max<int64_t>(tpi, nb));
  if (gmax < 1) return hipErrorInvalidValue;
  for (int64_t b0 = 0; b0 < a.batch; b0 += gmax) {
    const int g = (int)std::min<int64_t>(gmax, a.batch - b0);
    int* ea = (int*)ws;
    int* fb = ea + (int64_t)g * a.m;
    const hipError_t e = launch_group<S>(a, b0, g, ea, fb, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace emu8

hipError_t launch_emu8(const UniformArgs& a, int slices, void* ws, size_t ws_bytes,
                       hipStream_t s) {
  using namespace emu8;
  switch (slices) {
    case 1: return launch<1>(a, ws, ws_bytes, s);
    case 2: return launch<2>(a, ws, ws_bytes, s);
    case 3: return launch<3>(a, ws, ws_bytes, s);
    case 4: return launch<4>(a, ws, ws_bytes, s);
    case 5: return launch<5>(a, ws, ws_bytes, s);
    case 6: return launch<6>(a, ws, ws_bytes, s);
    case 7: return launch<7>(a, ws, ws_bytes, s);
    case 8: return launch<8>(a, ws, ws_bytes, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace bg
