// Batched FP64 GEMM kernels for CDNA4 (gfx950).
//
// Operation (the paper, Section II, Eq. 1): for every instance i,
//   C_i <- alpha * op(A_i) * op(B_i) + beta * C_i,   column-major, FP64.
// The paper builds each product from a 2-D grid of C tiles, one thread block
// per tile (Section II); here one workgroup computes one C tile with the
// 16x16x4 FP64 matrix-core instruction, operands staged through LDS.
//
// MFMA operand convention.  v_mfma_f64_16x16x4_f64 multiplies a 16x4 "A"
// fragment by a 4x16 "B" fragment.  Lane l holds element (l % 16, l / 16) of
// the A fragment and element (l / 16, l % 16) of the B fragment; result
// register v (v = 0..3) of lane l holds element (l / 16 + 4 v, l % 16) of the
// 16x16 result (checked on the device by the lane-layout test).  We feed
// op(B)^T as the instruction's A and op(A)^T as its B, so the result block is
// the transpose of a C block: lane l holds C(row = l % 16, col = l/16 + 4 v),
// i.e. 16 lanes cover 16 consecutive rows of one column -- the contiguous
// direction of column-major C, so epilogue loads/stores coalesce.
//
// Contraction-index permutation.  Within a 16-wide slice of k, MFMA number t
// (t = 0..3) uses k = kk + 4*g + t in lane group g = l / 16.  Any bijection of
// k is valid as long as both operands use it; this one lets a lane read four
// consecutive k values of a K-contiguous operand with one 32-byte LDS read.
#include "bgemm_internal.h"

namespace bg {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Tile configurations
// ---------------------------------------------------------------------------
template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NT = WAVES_M * WAVES_N * 64;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(BM % WM == 0 && BN % WN == 0 && WM % 16 == 0 && WN % 16 == 0, "tile");
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
};

using Cfg32 = Cfg<32, 32, 32, 32, 32>;
using Cfg64 = Cfg<64, 64, 32, 32, 32>;
using Cfg128 = Cfg<128, 128, 16, 64, 64>;

// ---------------------------------------------------------------------------
// Operand tiles.  An operand tile spans BMN values of its product dimension
// (m for A, n for B) and BK values of k.  In memory the operand is either
// MN-contiguous (A with 'N', B with 'T') or K-contiguous (A with 'T', B with
// 'N'); LDS keeps the memory orientation with a padded stride S (doubles):
//   MN-contiguous: lds[k * S + mn], S = BMN + 4  (S = 4 mod 8: the four lane
//                  groups of a fragment read land in distinct bank halves)
//   K-contiguous : lds[mn * S + k], S = BK + 2   (S = 2 mod 4: sixteen
//                  16-byte reads of one quarter-wave hit distinct banks)
// ---------------------------------------------------------------------------
template <int BMN, int BK, bool KC>
struct OpTile {
  static constexpr int LC = KC ? BK : BMN;  // extent along the contiguous dim
  static constexpr int LS = KC ? BMN : BK;  // extent along the strided dim
  static constexpr int S = KC ? BK + 2 : BMN + 4;
  static constexpr int ELEMS = LS * S;
};

template <class CF, bool TA, bool TB>
struct Smem {
  using TAt = OpTile<CF::BM, CF::BK, TA>;    // A is K-contiguous iff transposed
  using TBt = OpTile<CF::BN, CF::BK, !TB>;   // B is K-contiguous iff not transposed
  static constexpr int A_ELEMS = TAt::ELEMS, B_ELEMS = TBt::ELEMS;
  static constexpr int TOTAL = 2 * (A_ELEMS + B_ELEMS);  // double buffered
};

template <class CF>
struct SmemMax {
  static constexpr int a = Smem<CF, false, false>::TOTAL, b = Smem<CF, false, true>::TOTAL;
  static constexpr int c = Smem<CF, true, false>::TOTAL, d = Smem<CF, true, true>::TOTAL;
  static constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
  static constexpr int VALUE = ab > cd ? ab : cd;
};

// Global -> register -> LDS copy of one operand tile, NT threads, 16 bytes
// (two consecutive doubles along the contiguous dim) per thread per step.
template <int BMN, int BK, bool KC, int NT>
struct OpLoader {
  using T = OpTile<BMN, BK, KC>;
  static constexpr int PAIRS = T::LC * T::LS / 2;
  static constexpr int PER = PAIRS / NT;
  static_assert(PAIRS % NT == 0, "tile not divisible among threads");
  d2 v[PER];

  // base: operand matrix; ld: its leading dimension; (c0, s0): tile origin
  // along the contiguous / strided dims; (cext, sext): matrix extents there.
  __device__ __forceinline__ void load(const double* __restrict__ base, int64_t ld, int c0, int s0,
                                       int cext, int sext, bool fast, int tid) {
    if (fast) {
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        const int e = 2 * (tid + it * NT);
        const int cc = e % T::LC, ss = e / T::LC;
        v[it] = *reinterpret_cast<const d2*>(base + (c0 + cc) + (int64_t)(s0 + ss) * ld);
      }
    } else {
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        const int e = 2 * (tid + it * NT);
        const int cc = e % T::LC, ss = e / T::LC;
        const int c = c0 + cc, s = s0 + ss;
        const double* p = base + c + (int64_t)s * ld;
        const bool sok = s < sext;
        v[it].x = (sok && c < cext) ? p[0] : 0.0;
        v[it].y = (sok && c + 1 < cext) ? p[1] : 0.0;
      }
    }
  }

  __device__ __forceinline__ void store(double* lds, int tid) const {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = 2 * (tid + it * NT);
      const int cc = e % T::LC, ss = e / T::LC;
      *reinterpret_cast<d2*>(lds + ss * T::S + cc) = v[it];
    }
  }
};

// Reads this lane's fragments for NB 16-wide blocks starting at `mn0` and the
// 16-wide k slice starting at `kk`: f[b][t] = op(X)(mn0 + 16 b + l%16,
// kk + 4 (l/16) + t).
template <int BMN, int BK, bool KC, int NB>
__device__ __forceinline__ void read_frags(const double* lds, int mn0, int kk, int lane,
                                           double (&f)[NB][4]) {
  using T = OpTile<BMN, BK, KC>;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (KC) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const double* p = lds + (mn0 + 16 * b + r) * T::S + kk + 4 * g;
      const d2 lo = *reinterpret_cast<const d2*>(p);
      const d2 hi = *reinterpret_cast<const d2*>(p + 2);
      f[b][0] = lo.x; f[b][1] = lo.y; f[b][2] = hi.x; f[b][3] = hi.y;
    }
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) f[b][t] = lds[(kk + 4 * g + t) * T::S + mn0 + 16 * b + r];
  }
}

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

// ---------------------------------------------------------------------------
// One C tile (tm, tn) of one instance.  M, N, K are the sizes of op(A) (M x K)
// and op(B) (K x N).  use_product == false means alpha == 0 or K == 0: A and B
// are not read and C <- beta * C (exactly 0 when beta == 0, untouched when
// beta == 1).  Every thread of the workgroup must call this (it synchronises).
// ---------------------------------------------------------------------------
template <class CF, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(const double* __restrict__ A, int64_t lda,
                                          const double* __restrict__ B, int64_t ldb,
                                          double* __restrict__ C, int64_t ldc, int M, int N, int K,
                                          double alpha, double beta, int tm, int tn,
                                          double* lds) {
  using SM = Smem<CF, TA, TB>;
  using LA = OpLoader<CF::BM, CF::BK, TA, CF::NT>;
  using LB = OpLoader<CF::BN, CF::BK, !TB, CF::NT>;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % CF::WAVES_M) * CF::WM;
  const int wn0 = (wave / CF::WAVES_M) * CF::WN;
  const int m0 = tm * CF::BM, n0 = tn * CF::BN;
  const bool use_product = !(alpha == 0.0 || K == 0);

  d4 acc[CF::FM][CF::FN];
#pragma unroll
  for (int i = 0; i < CF::FM; ++i)
#pragma unroll
    for (int j = 0; j < CF::FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (use_product) {
    double* la[2] = {lds, lds + SM::A_ELEMS};
    double* lb[2] = {lds + 2 * SM::A_ELEMS, lds + 2 * SM::A_ELEMS + SM::B_ELEMS};
    // Extents of each operand along its (contiguous, strided) dims and the
    // origin of this tile along them for k-slice k0.
    const int a_cext = TA ? K : M, a_sext = TA ? M : K;
    const int b_cext = TB ? N : K, b_sext = TB ? K : N;
    const bool a_vec = aligned16(A) && (lda % 2 == 0);
    const bool b_vec = aligned16(B) && (ldb % 2 == 0);
    const bool a_mn_full = m0 + CF::BM <= M;
    const bool b_mn_full = n0 + CF::BN <= N;
    LA ra;
    LB rb;
    auto load = [&](int k0) {
      const bool kfull = k0 + CF::BK <= K;
      if (TA) ra.load(A, lda, k0, m0, a_cext, a_sext, a_vec && kfull && a_mn_full, tid);
      else    ra.load(A, lda, m0, k0, a_cext, a_sext, a_vec && kfull && a_mn_full, tid);
      if (TB) rb.load(B, ldb, n0, k0, b_cext, b_sext, b_vec && kfull && b_mn_full, tid);
      else    rb.load(B, ldb, k0, n0, b_cext, b_sext, b_vec && kfull && b_mn_full, tid);
    };
    const int nk = (K + CF::BK - 1) / CF::BK;
    load(0);
    ra.store(la[0], tid);
    rb.store(lb[0], tid);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) load((kt + 1) * CF::BK);
#pragma unroll
      for (int kk = 0; kk < CF::BK; kk += 16) {
        double fa[CF::FM][4], fb[CF::FN][4];
        read_frags<CF::BM, CF::BK, TA, CF::FM>(la[cur], wm0, kk, lane, fa);
        read_frags<CF::BN, CF::BK, !TB, CF::FN>(lb[cur], wn0, kk, lane, fb);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < CF::FM; ++i)
#pragma unroll
            for (int j = 0; j < CF::FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[j][t], fa[i][t], acc[i][j], 0, 0, 0);
      }
      if (kt + 1 < nk) {
        ra.store(la[cur ^ 1], tid);
        rb.store(lb[cur ^ 1], tid);
      }
      __syncthreads();
    }
  }

  // Epilogue: lane holds C(m0 + wm0 + 16 i + l%16, n0 + wn0 + 16 j + l/16 + 4 v).
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < CF::FM; ++i) {
    const int row = m0 + wm0 + 16 * i + r;
    if (row >= M) continue;
#pragma unroll
    for (int j = 0; j < CF::FN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = n0 + wn0 + 16 * j + g + 4 * v;
        if (col >= N) continue;
        double* p = C + row + (int64_t)col * ldc;
        if (use_product) {
          double x = alpha * acc[i][j][v];
          if (beta != 0.0) x = x + beta * (*p);
          *p = x;
        } else if (beta == 0.0) {
          *p = 0.0;
        } else if (beta != 1.0) {
          *p = beta * (*p);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Uniform batch: one workgroup per (instance, C tile).  Workgroups are handed
// to the eight XCDs round-robin by id, so id -> (instance, tile) is remapped
// to give each XCD a contiguous range of tiles: all tiles of an instance run
// on one XCD at about the same time and share its L2 for the A/B panels.
// ---------------------------------------------------------------------------
constexpr int NUM_XCD = 8;

template <class CF, bool TA, bool TB>
__global__ __launch_bounds__(CF::NT) void k_uniform(
    int M, int N, int K, double alpha, const double* const* __restrict__ Ap, int64_t lda,
    const double* const* __restrict__ Bp, int64_t ldb, double beta,
    double* const* __restrict__ Cp, int64_t ldc, int tiles_m, int tiles_per_inst,
    int64_t total_tiles, int64_t per_xcd) {
  __shared__ double lds[SmemMax<CF>::VALUE];
  const int64_t bid = blockIdx.x;
  const int64_t id = (bid % NUM_XCD) * per_xcd + bid / NUM_XCD;
  if (id >= total_tiles) return;
  const int64_t inst = id / tiles_per_inst;
  const int t = (int)(id - inst * tiles_per_inst);
  const int tm = t % tiles_m, tn = t / tiles_m;
  gemm_tile<CF, TA, TB>(Ap[inst], lda, Bp[inst], ldb, Cp[inst], ldc, M, N, K, alpha, beta, tm,
                        tn, lds);
}

template <class CF, bool TA, bool TB>
static hipError_t launch_uniform_t(const UniformArgs& a, hipStream_t s) {
  const int tiles_m = (a.m + CF::BM - 1) / CF::BM;
  const int tiles_n = (a.n + CF::BN - 1) / CF::BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int64_t total = tpi * a.batch;
  if (tpi > INT32_MAX) return hipErrorInvalidValue;
  const int64_t per_xcd = (total + NUM_XCD - 1) / NUM_XCD;
  const int64_t grid = per_xcd * NUM_XCD;
  if (grid > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_uniform<CF, TA, TB>), dim3((unsigned)grid), dim3(CF::NT), 0, s, a.m, a.n,
                     a.k, a.alpha, a.A, a.lda, a.B, a.ldb, a.beta, a.C, a.ldc, tiles_m, (int)tpi,
                     total, per_xcd);
  return hipGetLastError();
}

template <class CF>
static hipError_t launch_uniform_c(const UniformArgs& a, hipStream_t s) {
  if (!a.ta && !a.tb) return launch_uniform_t<CF, false, false>(a, s);
  if (!a.ta && a.tb) return launch_uniform_t<CF, false, true>(a, s);
  if (a.ta && !a.tb) return launch_uniform_t<CF, true, false>(a, s);
  return launch_uniform_t<CF, true, true>(a, s);
}

TileShape tile_shape(TileClass c) {
  switch (c) {
    case TC_32: return {Cfg32::BM, Cfg32::BN, Cfg32::BK, Cfg32::NT};
    case TC_64: return {Cfg64::BM, Cfg64::BN, Cfg64::BK, Cfg64::NT};
    default: return {Cfg128::BM, Cfg128::BN, Cfg128::BK, Cfg128::NT};
  }
}

TileClass pick_uniform_class(int m, int n, int k, int force) {
  (void)k;
  if (force >= 0 && force < TC_COUNT) return (TileClass)force;
  const int mx = m > n ? m : n;
  if (mx <= 32) return TC_32;
  if (mx <= 64) return TC_64;
  return TC_128;
}

hipError_t launch_uniform(const UniformArgs& a, TileClass cls, hipStream_t s) {
  switch (cls) {
    case TC_32: return launch_uniform_c<Cfg32>(a, s);
    case TC_64: return launch_uniform_c<Cfg64>(a, s);
    default: return launch_uniform_c<Cfg128>(a, s);
  }
}

// C_i <- beta * C_i, or exactly 0 when beta == 0 (C not read).
__global__ __launch_bounds__(256) void k_scale(double beta, double* const* __restrict__ Cp,
                                               int64_t ldc, int m, int n, int64_t total_cols) {
  for (int64_t col = blockIdx.x; col < total_cols; col += gridDim.x) {
    const int64_t inst = col / n;
    const int j = (int)(col - inst * n);
    double* p = Cp[inst] + (int64_t)j * ldc;
    for (int r = threadIdx.x; r < m; r += blockDim.x) p[r] = (beta == 0.0) ? 0.0 : beta * p[r];
  }
}

hipError_t launch_scale(double beta, double* const* C, int64_t ldc, int m, int n, int batch,
                        hipStream_t s) {
  const int64_t cols = (int64_t)n * batch;
  const int64_t grid = cols < 65536 ? cols : 65536;
  hipLaunchKernelGGL(k_scale, dim3((unsigned)grid), dim3(256), 0, s, beta, C, ldc, m, n, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Variable-size batch (the paper, Section II: each GEMM gets its own 2-D grid
// of tiles, sizes differ per instance).  Sizes live on the device, so the
// whole plan is made there:
//   1. k_vb_count: validate each instance (info), count its C tiles, and
//      scan the counts within each block of 256 instances;
//   2. k_vb_blocks: scan the block totals (one workgroup), reset the queue;
//   3. k_vb_finish: global exclusive prefix P[i] and, when it fits, a map
//      tile -> instance;
//   4. k_vb_exec: a persistent grid; each workgroup pops tile numbers from an
//      atomic counter until the queue is empty.
// ---------------------------------------------------------------------------
using CfgVb = Cfg64;
constexpr int PLAN_BLOCK = 256;

struct VbLayout {
  int64_t* prefix;   // [batch + 1]
  int64_t* bsum;     // [nblocks]
  int64_t* ctrl;     // [0] total tiles, [1] queue head
  int* map;          // [map_cap]
  int64_t map_cap;
};

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t vbatched_workspace_bytes(int batch) {
  const size_t nb = ((size_t)batch + PLAN_BLOCK - 1) / PLAN_BLOCK;
  return align256(((size_t)batch + 1) * 8) + align256(nb * 8) + align256(64);
}

static VbLayout vb_layout(const VbWorkspace& ws, int batch) {
  VbLayout L;
  char* p = (char*)ws.base;
  const size_t nb = ((size_t)batch + PLAN_BLOCK - 1) / PLAN_BLOCK;
  L.prefix = (int64_t*)p; p += align256(((size_t)batch + 1) * 8);
  L.bsum = (int64_t*)p; p += align256(nb * 8);
  L.ctrl = (int64_t*)p; p += align256(64);
  const size_t used = (size_t)(p - (char*)ws.base);
  L.map = (int*)p;
  L.map_cap = used < ws.bytes ? (int64_t)((ws.bytes - used) / sizeof(int)) : 0;
  return L;
}

// Argument numbers follow reference-BLAS DGEMM (3 m, 4 n, 5 k, 8 lda, 10 ldb,
// 13 ldc).  Returns 0 for a valid instance.
__device__ __forceinline__ int vb_check(bool ta, bool tb, int m, int n, int k, int lda, int ldb,
                                        int ldc) {
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  const int ra = ta ? k : m, rb = tb ? n : k;
  if (lda < (ra > 1 ? ra : 1)) return -8;
  if (ldb < (rb > 1 ? rb : 1)) return -10;
  if (ldc < (m > 1 ? m : 1)) return -13;
  return 0;
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_count(
    bool ta, bool tb, const int* __restrict__ m, const int* __restrict__ n,
    const int* __restrict__ k, const int* __restrict__ lda, const int* __restrict__ ldb,
    const int* __restrict__ ldc, double alpha, double beta, int batch, int* __restrict__ info,
    int64_t* __restrict__ prefix, int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[PLAN_BLOCK];
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  int64_t tiles = 0;
  if (i < batch) {
    const int mi = m[i], ni = n[i], ki = k[i];
    const int st = vb_check(ta, tb, mi, ni, ki, lda[i], ldb[i], ldc[i]);
    if (info) info[i] = st;
    const bool noop = (alpha == 0.0 || ki == 0) && beta == 1.0;
    if (st == 0 && mi > 0 && ni > 0 && !noop)
      tiles = (int64_t)((mi + CfgVb::BM - 1) / CfgVb::BM) * ((ni + CfgVb::BN - 1) / CfgVb::BN);
  }
  // inclusive scan within the block (Hillis-Steele in LDS)
  sh[threadIdx.x] = tiles;
  __syncthreads();
  for (int off = 1; off < PLAN_BLOCK; off <<= 1) {
    const int64_t x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  if (i < batch) prefix[i] = sh[threadIdx.x] - tiles;  // exclusive, block-local
  if (threadIdx.x == PLAN_BLOCK - 1) bsum[blockIdx.x] = sh[PLAN_BLOCK - 1];
}

__global__ __launch_bounds__(1024) void k_vb_blocks(int64_t* __restrict__ bsum, int nblocks,
                                                    int64_t* __restrict__ ctrl) {
  // exclusive scan of bsum in place, 1024 values per pass, carrying the sum
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nblocks; base += 1024) {
    const int i = base + threadIdx.x;
    const int64_t x = i < nblocks ? bsum[i] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nblocks) bsum[i] = carry + sh[threadIdx.x] - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ctrl[0] = carry;  // total tiles
    ctrl[1] = 0;      // queue head
  }
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_finish(int batch, int64_t* __restrict__ prefix,
                                                          const int64_t* __restrict__ bsum,
                                                          const int64_t* __restrict__ ctrl) {
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  if (i >= batch) return;
  prefix[i] += bsum[blockIdx.x];
  if (i == batch - 1) prefix[batch] = ctrl[0];
}

// Writes the tile -> instance map once all prefixes are final.
__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_map(int batch, const int64_t* __restrict__ prefix,
                                                       const int64_t* __restrict__ ctrl,
                                                       int* __restrict__ map, int64_t map_cap) {
  const int64_t total = ctrl[0];
  if (total > map_cap) return;
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  if (i >= batch) return;
  const int64_t lo = prefix[i], hi = prefix[i + 1];
  for (int64_t t = lo; t < hi; ++t) map[t] = i;
}

// Instance owning tile q: the last i with prefix[i] <= q (and prefix[i+1] > q).
__device__ __forceinline__ int vb_find(const int64_t* __restrict__ prefix, int batch, int64_t q) {
  int lo = 0, hi = batch;  // invariant: prefix[lo] <= q < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(CfgVb::NT) void k_vb_exec(
    const int* __restrict__ m, const int* __restrict__ n, const int* __restrict__ k, double alpha,
    const double* const* __restrict__ Ap, const int* __restrict__ lda,
    const double* const* __restrict__ Bp, const int* __restrict__ ldb, double beta,
    double* const* __restrict__ Cp, const int* __restrict__ ldc, int batch,
    const int64_t* __restrict__ prefix, int64_t* __restrict__ ctrl, const int* __restrict__ map,
    int64_t map_cap) {
  __shared__ double lds[SmemMax<CfgVb>::VALUE];
  __shared__ int64_t s_q;
  const int64_t total = ctrl[0];
  const bool use_map = total <= map_cap;
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd((unsigned long long*)&ctrl[1], 1ull);
    __syncthreads();
    const int64_t q = s_q;
    __syncthreads();
    if (q >= total) break;
    const int i = use_map ? map[q] : vb_find(prefix, batch, q);
    const int mi = m[i], ni = n[i], ki = k[i];
    const int tiles_m = (mi + CfgVb::BM - 1) / CfgVb::BM;
    const int t = (int)(q - prefix[i]);
    gemm_tile<CfgVb, TA, TB>(Ap[i], lda[i], Bp[i], ldb[i], Cp[i], ldc[i], mi, ni, ki, alpha, beta,
                             t % tiles_m, t / tiles_m, lds);
  }
}

hipError_t launch_vbatched(const VbatchedArgs& a, const VbWorkspace& ws, int num_cus,
                           hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  if (vbatched_workspace_bytes(a.batch) > ws.bytes) return hipErrorOutOfMemory;
  const VbLayout L = vb_layout(ws, a.batch);
  const int nb = (a.batch + PLAN_BLOCK - 1) / PLAN_BLOCK;
  hipLaunchKernelGGL(k_vb_count, dim3(nb), dim3(PLAN_BLOCK), 0, s, a.ta, a.tb, a.m, a.n, a.k, a.lda,
                     a.ldb, a.ldc, a.alpha, a.beta, a.batch, a.info, L.prefix, L.bsum);
  hipLaunchKernelGGL(k_vb_blocks, dim3(1), dim3(1024), 0, s, L.bsum, nb, L.ctrl);
  hipLaunchKernelGGL(k_vb_finish, dim3(nb), dim3(PLAN_BLOCK), 0, s, a.batch, L.prefix, L.bsum,
                     L.ctrl);
  hipLaunchKernelGGL(k_vb_map, dim3(nb), dim3(PLAN_BLOCK), 0, s, a.batch, L.prefix, L.ctrl, L.map,
                     L.map_cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  int per_cu = 0;
  auto kern = a.ta ? (a.tb ? k_vb_exec<true, true> : k_vb_exec<true, false>)
                   : (a.tb ? k_vb_exec<false, true> : k_vb_exec<false, false>);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, CfgVb::NT, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int grid = num_cus * per_cu;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(CfgVb::NT), 0, s, a.m, a.n, a.k, a.alpha, a.A, a.lda,
                     a.B, a.ldb, a.beta, a.C, a.ldc, a.batch, L.prefix, L.ctrl, L.map, L.map_cap);
  return hipGetLastError();
}

}  // namespace bg
