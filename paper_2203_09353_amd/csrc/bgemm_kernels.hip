// Batched FP64 GEMM kernels for CDNA4 (gfx950).
//
// Operation (the paper, Section II, Eq. 1): for every instance i,
//   C_i <- alpha * op(A_i) * op(B_i) + beta * C_i,   column-major, FP64.
// The paper builds each product from a 2-D grid of C tiles, one thread block
// per tile (Section II); here one workgroup computes one C tile on the FP64
// matrix cores, operands staged through LDS.
//
// Matrix-core instruction.  v_mfma_f64_4x4x4_4b_f64 performs four independent
// 4x4x4 products per wave (blocks b = 0..3).  Lane 16 s + 4 b + i holds
// element (i, s) of block b's first operand, lane 16 s + 4 b + j holds element
// (s, j) of its second operand, and the result element (i, j) of block b lands
// in lane 16 i + 4 b + j (checked on the device by the lane-layout test).  On
// gfx950 this instruction sustains about 1.5x the FP64 rate of the 16x16x4
// form, so the tiles are built from it.
//
// Roles.  Of the two operands of the product, one -- "P" -- is read as a
// 16-row slab: lane 16 s + r holds P(p0 + r, k_s), so the four blocks cover
// 16 consecutive P indices.  The other -- "Q" -- is read replicated: lane
// 16 s + 4 b + j holds Q(q0 + j, k_s) for every b.  One instruction then
// yields a 16 x 4 block of P x Q^T: lane 16 i + 4 b + j holds the sum over s
// of P(p0 + 4 b + i, k_s) Q(q0 + j, k_s).  With P = op(A) and Q = op(B)^T the
// block is a piece of C whose 16 rows sit in 16 lanes (coalesced column
// segments); with P = op(B)^T and Q = op(A) it is a piece of C^T.  The larger
// tiles use the second form because it needs less LDS padding.
//
// Contraction order.  A 16-wide slice of k starting at kk is consumed by four
// instructions t = 0..3; instruction t gives lane group s the index
// k = kk + 2 s + 8 (t / 2) + (t % 2).  Any bijection is valid if both operands
// use it; this one puts each t-pair on adjacent k, so a K-contiguous operand
// feeds two instructions with one 16-byte LDS read.  Every tile class walks k
// in the same slices and order, so a given element of C gets the same bits
// from every class, alone or in any batch.
#include <type_traits>

#include "bgemm_internal.h"

namespace bg {

typedef double d2 __attribute__((ext_vector_type(2)));
// a pair of doubles at any 8-byte boundary: with an odd leading dimension
// every other column's pairs start off a 16-byte boundary, and the memory
// system serves such 16-byte accesses (unaligned access mode)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// Explicit address spaces: matrices are global memory (address space 1),
// operand tiles are LDS (address space 3).  Without them the compiler falls
// back to flat instructions, which count against both the vector-memory and
// the LDS wait counters and so serialise LDS reads behind global prefetches.
#define AS_GLOBAL __attribute__((address_space(1)))
#define AS_LDS __attribute__((address_space(3)))
typedef const AS_GLOBAL double* gcptr;
typedef AS_GLOBAL double* gptr;
typedef AS_LDS double* lptr;
typedef const AS_LDS double* lcptr;

// Accesses to C on interior tiles.  A tile reads its part of C once and
// writes it once, so these are nontemporal: the 200,000 x 64^3 batch (half of
// its bytes are C reads and writes) runs 2.5-3.5 % faster, 256^3 0.1-0.7 %,
// the variable-size batch within noise.  Edge tiles keep ordinary accesses
// (nontemporal there made the variable-size batch 0.5 % slower), and so do
// the operand loads (nontemporal A and B loads were faster still on 64^3 but
// made the variable-size batch 7 % slower: its tiles share A and B panels
// through the caches).
#ifndef BG_NT_C
#define BG_NT_C 1
#endif
template <class T>
__device__ __forceinline__ T ld_c(const AS_GLOBAL T* p) {
  if constexpr (BG_NT_C) return __builtin_nontemporal_load(p);
  else return *p;
}
template <class T>
__device__ __forceinline__ void st_c(AS_GLOBAL T* p, T v) {
  if constexpr (BG_NT_C) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// ---------------------------------------------------------------------------
// Tile configurations: C tile BM x BN per workgroup, BK of k per LDS stage,
// wave tile WM x WN, SWAP selects the C^T form (P = op(B)^T, Q = op(A)).
// ---------------------------------------------------------------------------
template <int BM_, int BN_, int BK_, int WM_, int WN_, bool SWAP_, int NSTAGE_ = 2,
          bool CPRE_ = false, int SKIP_ = 0, int PIPE_ = 0>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr bool SWAP = SWAP_;
  static constexpr int NSTAGE = NSTAGE_;      // LDS buffers (2: double buffered)
  static constexpr bool CPRE = CPRE_;         // read C (beta != 0) before the k loop
  // Work skipped on edge tiles: 0 none, 1 waves whose region lies outside C
  // (on the pipelined path also the 16-wide P slabs outside C), 2 on the
  // register path also single instructions whose 16 x 4 output lies outside
  // C.
  static constexpr int SKIP = SKIP_;
  // PIPE >= 3: instances whose A and B are 16-byte aligned with even leading
  // dimensions use the pipelined path, a ring of PIPE LDS stages filled by
  // direct global-to-LDS loads; 0 disables it.
  static constexpr int PIPE = PIPE_;
  static_assert(PIPE == 0 || PIPE >= 3, "the pipelined path needs at least three stages");
  static_assert(NSTAGE == 1 || NSTAGE == 2, "one or two LDS stages");
  static constexpr int WAVES_M = BM / WM, WAVES_N = BN / WN;
  static constexpr int NT = WAVES_M * WAVES_N * 64;
  static constexpr int WP = SWAP ? WN : WM;   // wave extent along P
  static constexpr int WQ = SWAP ? WM : WN;   // wave extent along Q
  static constexpr int FP = WP / 16;          // 16-wide P slabs per wave
  static constexpr int GQ = WQ / 4;           // 4-wide Q groups per wave
  static_assert(BM % WM == 0 && BN % WN == 0 && WP % 16 == 0 && WQ % 4 == 0, "tile");
  static_assert(BK % 16 == 0, "BK must be a multiple of 16");
};

// Shapes per size class (BM, BN, BK, WM, WN, SWAP); the BG_CFG* macros let a
// tuning build try other shapes without editing the source.
#ifndef BG_CFG32
#define BG_CFG32 32, 32, 32, 32, 32, false
#endif
#ifndef BG_CFG64
#define BG_CFG64 64, 64, 16, 32, 32, true, 2, true
#endif
#ifndef BG_CFG128
#define BG_CFG128 128, 64, 16, 16, 64, true, 2, false, 0, 3
#endif
// Guarded loads as unconditional loads from clamped addresses plus a select
// (1), or as predicated loads (0).
#ifndef BG_CLAMPED_LOADS
#define BG_CLAMPED_LOADS 0
#endif
// The pipelined path for any 8-byte-aligned operands and any leading
// dimension (1: a 16-byte unit then starts at an 8-byte boundary whenever a
// column starts at one), or only for 16-byte-aligned operands with even
// leading dimensions (0).
#ifndef BG_PIPE_ANY_LD
#define BG_PIPE_ANY_LD 1
#endif
// Pipelined path: a k-step's refill loads issued after its first 16-slice's
// second fragment read (1: their address arithmetic overlaps the LDS reads
// and the first products), or right after the barrier (0).
#ifndef BG_PIPE_LATE_REFILL
#define BG_PIPE_LATE_REFILL 1
#endif
// Pipelined path: wave priority raised from a k-step's barrier to its end
// (1), or left at 0.
#ifndef BG_PIPE_SETPRIO
#define BG_PIPE_SETPRIO 1
#endif
// Epilogue C loads all issued before the stores (1), or per element (0).
#ifndef BG_EPI_BATCH
#define BG_EPI_BATCH 1
#endif
using Cfg32 = Cfg<BG_CFG32>;
using Cfg64 = Cfg<BG_CFG64>;
using Cfg128 = Cfg<BG_CFG128>;

// ---------------------------------------------------------------------------
// Operand tiles in LDS.  An operand tile spans BMN values of its product
// dimension (m for A, n for B) and BK values of k.  In memory the operand is
// MN-contiguous (A with 'N', B with 'T') or K-contiguous (A with 'T', B with
// 'N'); LDS keeps that orientation with a padded stride S (doubles), chosen
// per role so that one read instruction hits distinct banks (64 banks of
// 4 bytes):
//   P, MN-contiguous lds[k*S + mn]: S = BMN + 8  (4 S = 32 mod 64: lane
//      groups s = 0, 1 fall in opposite bank halves)
//   P, K-contiguous  lds[mn*S + k]: S = BK + 2   (2 S = 4 mod 8: sixteen
//      16-byte reads of a quarter-wave are disjoint)
//   Q, MN-contiguous lds[k*S + mn]: S = BMN + 2  (4 S = 8 mod 64)
//   Q, K-contiguous  lds[mn*S + k]: S = BK + 8   (2 S = 16 or 48 mod 64: the
//      four columns read by a quarter-wave are 16 banks apart)
// ---------------------------------------------------------------------------
template <int BMN, int BK, bool KC, bool ROLE_P>
struct OpTile {
  static constexpr int LC = KC ? BK : BMN;  // extent along the contiguous dim
  static constexpr int LS = KC ? BMN : BK;  // extent along the strided dim
  static constexpr int S = KC ? (ROLE_P ? BK + 2 : BK + 8) : (ROLE_P ? BMN + 8 : BMN + 2);
  static constexpr int ELEMS = LS * S;
};

// A is K-contiguous iff transposed; B is K-contiguous iff not transposed.
template <class CF, bool TA, bool TB>
struct Smem {
  using TAt = OpTile<CF::BM, CF::BK, TA, !CF::SWAP>;
  using TBt = OpTile<CF::BN, CF::BK, !TB, CF::SWAP>;
  static constexpr int A_ELEMS = TAt::ELEMS, B_ELEMS = TBt::ELEMS;
  static constexpr int TOTAL = CF::NSTAGE * (A_ELEMS + B_ELEMS);
};


// Global -> register -> LDS copy of one operand tile, NT threads, 16 bytes
// (two consecutive doubles along the contiguous dim) per thread per step.
template <class T, int NT>
struct OpLoader {
  static constexpr int PAIRS = T::LC * T::LS / 2;
  static constexpr int PER = PAIRS / NT;
  static_assert(PAIRS % NT == 0, "tile not divisible among threads");
  d2 v[PER];

  // base: operand matrix; ld: its leading dimension; (c0, s0): tile origin
  // along the contiguous / strided dims; (cext, sext): matrix extents there.
  // `fast`: the whole tile is inside the matrix.
  __device__ __forceinline__ void load(gcptr base, int64_t ld, int c0, int s0, int cext, int sext,
                                       bool fast, int tid) {
    if (fast) {
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        const int e = 2 * (tid + it * NT);
        const int cc = e % T::LC, ss = e / T::LC;
        v[it] = *(const AS_GLOBAL d2u*)(base + (c0 + cc) + (int64_t)(s0 + ss) * ld);
      }
    } else {
#pragma unroll
      for (int it = 0; it < PER; ++it) {
        const int e = 2 * (tid + it * NT);
        const int cc = e % T::LC, ss = e / T::LC;
        const int c = c0 + cc, s = s0 + ss;
        const bool sok = s < sext;
        if (BG_CLAMPED_LOADS) {
          // unconditional loads from clamped (in-bounds) addresses, then a
          // select: no branch around each load, so all of them are in flight
          const int64_t col = (int64_t)(sok ? s : sext - 1) * ld;
          const double x0 = base[(c < cext ? c : cext - 1) + col];
          const double x1 = base[(c + 1 < cext ? c + 1 : cext - 1) + col];
          v[it].x = (sok && c < cext) ? x0 : 0.0;
          v[it].y = (sok && c + 1 < cext) ? x1 : 0.0;
        } else {
          const gcptr p = base + c + (int64_t)s * ld;
          v[it].x = (sok && c < cext) ? p[0] : 0.0;
          v[it].y = (sok && c + 1 < cext) ? p[1] : 0.0;
        }
      }
    }
  }

  __device__ __forceinline__ void store(lptr lds, int tid) const {
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = 2 * (tid + it * NT);
      const int cc = e % T::LC, ss = e / T::LC;
      *(AS_LDS d2*)(lds + ss * T::S + cc) = v[it];
    }
  }
};

// k offset (within a 16-slice) of lane group s for instruction t.
__device__ __forceinline__ int kperm(int s, int t) { return 2 * s + 8 * (t >> 1) + (t & 1); }

// P-role fragments of NB slabs for the instruction pair (2 tp, 2 tp + 1):
// f[b][u] = X(mn0 + 16 b + l%16, kk + kperm(l/16, 2 tp + u)).
template <class T, int NB, bool KC>
__device__ __forceinline__ void read_p(lcptr lds, int mn0, int kk, int tp, int lane,
                                       double (&f)[NB][2]) {
  const int r = lane & 15, s = lane >> 4;
  const int k = kk + 2 * s + 8 * tp;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (KC) {
      const d2 x = *(const AS_LDS d2*)(lds + (mn0 + 16 * b + r) * T::S + k);
      f[b][0] = x.x; f[b][1] = x.y;
    } else {
      f[b][0] = lds[k * T::S + mn0 + 16 * b + r];
      f[b][1] = lds[(k + 1) * T::S + mn0 + 16 * b + r];
    }
  }
}

// Q-role fragments of NG groups: f[g][u] = X(mn0 + 4 g + l%4, kk + kperm(l/16, 2 tp + u)).
template <class T, int NG, bool KC>
__device__ __forceinline__ void read_q(lcptr lds, int mn0, int kk, int tp, int lane,
                                       double (&f)[NG][2]) {
  const int j = lane & 3, s = lane >> 4;
  const int k = kk + 2 * s + 8 * tp;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if constexpr (KC) {
      const d2 x = *(const AS_LDS d2*)(lds + (mn0 + 4 * g + j) * T::S + k);
      f[g][0] = x.x; f[g][1] = x.y;
    } else {
      f[g][0] = lds[k * T::S + mn0 + 4 * g + j];
      f[g][1] = lds[(k + 1) * T::S + mn0 + 4 * g + j];
    }
  }
}

// ---------------------------------------------------------------------------
// Pipelined path: operand tiles without padding, 16-byte units XOR-swizzled
// within each row so that the same fragment reads as above stay on distinct
// banks.  A row is one step of the strided dimension (a column of an
// MN-contiguous operand, a k-row of a K-contiguous one... in LDS terms: LS rows
// of UR = LC / 2 units).  Unit u of row r sits at r * UR + (u ^ sw(r)):
//   K-contiguous  (LC = BK): sw = (r / 2) mod 8 when UR = 8, else r mod 16 --
//      sixteen rows read at the same unit land in sixteen distinct 16-byte
//      bank groups;
//   MN-contiguous (LC = BMN): sw = 8 * ((r / 2) mod 2) -- rows k and k + 2,
//      read by the two lane groups of a half-wave, fall in opposite halves.
// A direct load (global_load_lds_dwordx4) writes 64 consecutive units (1 KB)
// per wave instruction, lane l at unit l; so each lane fetches the global pair
// that the swizzle places at its unit.
// ---------------------------------------------------------------------------
template <int BMN, int BK, bool KC>
struct SwTile {
  static constexpr int LC = KC ? BK : BMN;
  static constexpr int LS = KC ? BMN : BK;
  static constexpr int UR = LC / 2;
  static constexpr int UNITS = UR * LS;
  static constexpr int ELEMS = 2 * UNITS;
  static_assert((UR & (UR - 1)) == 0 && UR >= 8, "rows of a power-of-two number of units >= 8");
  static_assert(UNITS % 64 == 0, "whole 1 KB chunks");
  __device__ __forceinline__ static int sw(int r) {
    if constexpr (KC) return UR == 8 ? ((r >> 1) & 7) : (r & 15);
    else return ((r >> 1) & 1) << 3;
  }
  // offset (doubles) of logical element (row r, contiguous index c)
  __device__ __forceinline__ static int off(int r, int c) {
    return 2 * (r * UR + ((c >> 1) ^ sw(r))) + (c & 1);
  }
};

// Issues the direct loads of one operand tile (origin c0 / s0 along the
// contiguous / strided dims, extents cext / sext; the origin is inside the
// matrix).  Units outside the matrix read the tile's first pair instead (their
// products only reach C elements outside the matrix, which are never stored);
// k beyond K never reaches this path.  A pair straddling an odd cext reads one element of ld padding, which
// exists because ld is even; the last column, where that could leave the
// allocation, is always loaded by tail_tile.
template <class T, int NT>
__device__ __forceinline__ void dma_tile(gcptr base, int64_t ld, int c0, int s0, int cext,
                                         int sext, lptr dst, int wave, int lane) {
  constexpr int NW = NT / 64;
  constexpr int CH = T::UNITS / 64;
  static_assert(CH % NW == 0, "chunks not divisible among waves");
#pragma unroll
  for (int it = 0; it < CH / NW; ++it) {
    const int chunk = it * NW + wave;
    const int unit = chunk * 64 + lane;
    const int r = unit / T::UR, pu = unit % T::UR;
    int c = c0 + 2 * (pu ^ T::sw(r));
    int sr = s0 + r;
    // Lanes outside the matrix re-read the tile's first pair (in bounds, same
    // cache lines).  Every wave must issue exactly the same number of direct
    // loads per step -- the stage waits count them -- so lanes are never
    // masked off: a wave whose lanes were all masked would skip the
    // instruction.
    c = c < cext ? c : c0;
    sr = sr < sext ? sr : s0;
    __builtin_amdgcn_global_load_lds((const AS_GLOBAL void*)(base + c + (int64_t)sr * ld),
                                     (AS_LDS void*)(dst + chunk * 128), 16, 0, 0);
  }
}

// Guarded copy of one operand tile through registers, zero outside the
// matrix; used for the last k-step (partial in k, or holding the last column
// of an odd-extent MN-contiguous operand).
template <class T, int NT>
__device__ __forceinline__ void tail_tile(gcptr base, int64_t ld, int c0, int s0, int cext,
                                          int sext, lptr dst, int tid) {
  static_assert(T::UNITS % NT == 0, "whole rounds");
#pragma unroll
  for (int e = tid; e < T::UNITS; e += NT) {
    const int r = e / T::UR, u = e % T::UR;
    const int c = c0 + 2 * u, sr = s0 + r;
    const bool ok = sr < sext;
    d2 v;
    if (BG_CLAMPED_LOADS) {
      const int64_t col = (int64_t)(ok ? sr : sext - 1) * ld;
      const double x0 = base[(c < cext ? c : cext - 1) + col];
      const double x1 = base[(c + 1 < cext ? c + 1 : cext - 1) + col];
      v.x = (ok && c < cext) ? x0 : 0.0;
      v.y = (ok && c + 1 < cext) ? x1 : 0.0;
    } else {
      const gcptr p = base + c + (int64_t)sr * ld;
      v.x = (ok && c < cext) ? p[0] : 0.0;
      v.y = (ok && c + 1 < cext) ? p[1] : 0.0;
    }
    *(AS_LDS d2*)(dst + T::off(r, 2 * u)) = v;
  }
}

// Fragment reads from swizzled tiles; same lane / index convention as
// read_p / read_q.
template <class T, int NB, bool KC>
__device__ __forceinline__ void read_p_sw(lcptr lds, int mn0, int kk, int tp, int lane,
                                          double (&f)[NB][2]) {
  const int r = lane & 15, s = lane >> 4;
  const int k = kk + 2 * s + 8 * tp;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (KC) {
      const d2 x = *(const AS_LDS d2*)(lds + T::off(mn0 + 16 * b + r, k));
      f[b][0] = x.x; f[b][1] = x.y;
    } else {
      f[b][0] = lds[T::off(k, mn0 + 16 * b + r)];
      f[b][1] = lds[T::off(k + 1, mn0 + 16 * b + r)];
    }
  }
}

template <class T, int NG, bool KC>
__device__ __forceinline__ void read_q_sw(lcptr lds, int mn0, int kk, int tp, int lane,
                                          double (&f)[NG][2]) {
  const int j = lane & 3, s = lane >> 4;
  const int k = kk + 2 * s + 8 * tp;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if constexpr (KC) {
      const d2 x = *(const AS_LDS d2*)(lds + T::off(mn0 + 4 * g + j, k));
      f[g][0] = x.x; f[g][1] = x.y;
    } else {
      f[g][0] = lds[T::off(k, mn0 + 4 * g + j)];
      f[g][1] = lds[T::off(k + 1, mn0 + 4 * g + j)];
    }
  }
}

// s_waitcnt immediate: vector-memory count vm, LDS/scalar count lgkm, export
// count unconstrained (gfx9 encoding).
constexpr int waitcnt_imm(int vm, int lgkm) {
  return (vm & 15) | ((vm >> 4) << 14) | (7 << 4) | ((lgkm & 15) << 8);
}

template <class CF, bool TA, bool TB>
struct PipeSmem {
  using TAs = SwTile<CF::BM, CF::BK, TA>;
  using TBs = SwTile<CF::BN, CF::BK, !TB>;
  static constexpr int STAGE = TAs::ELEMS + TBs::ELEMS;
  static constexpr int TOTAL = CF::PIPE * STAGE;
  // direct loads per thread per k-step
  static constexpr int DPT = (TAs::UNITS + TBs::UNITS) / CF::NT;
};

// LDS of a kernel that may take either path for a tile
template <class CF, bool TA, bool TB>
struct TileSmem {
  static constexpr int a = Smem<CF, TA, TB>::TOTAL;
  static constexpr int b = CF::PIPE ? PipeSmem<CF, TA, TB>::TOTAL : 0;
  static constexpr int TOTAL = a > b ? a : b;
};

__device__ __forceinline__ bool aligned16(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}
__device__ __forceinline__ bool aligned8(const void* p) {
  return (reinterpret_cast<uintptr_t>(p) & 7) == 0;
}

// ---------------------------------------------------------------------------
// One C tile (tm, tn) of one instance.  M, N, K are the sizes of op(A) (M x K)
// and op(B) (K x N).  use_product == false means alpha == 0 or K == 0: A and B
// are not read and C <- beta * C (exactly 0 when beta == 0, untouched when
// beta == 1).  Every thread of the workgroup must call this (it synchronises).
// ---------------------------------------------------------------------------
template <class CF, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(const double* A_, int64_t lda, const double* B_,
                                          int64_t ldb, double* C_, int64_t ldc, int M, int N, int K,
                                          double alpha, double beta, int tm, int tn, lptr lds) {
  const gcptr A = (gcptr)A_;
  const gcptr B = (gcptr)B_;
  const gptr C = (gptr)C_;
  using SM = Smem<CF, TA, TB>;
  using TAt = typename SM::TAt;
  using TBt = typename SM::TBt;
  using LA = OpLoader<TAt, CF::NT>;
  using LB = OpLoader<TBt, CF::NT>;
  constexpr bool SW = CF::SWAP;
  // The thread id passes through an opaque move, so that the lane-dependent
  // LDS and global offsets below are computed inside this tile rather than
  // hoisted out of a persistent caller's tile loop, where they would stay
  // live (in registers) across every tile.
  int tid;
  asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % CF::WAVES_M) * CF::WM;
  const int wn0 = (wave / CF::WAVES_M) * CF::WN;
  const int m0 = tm * CF::BM, n0 = tn * CF::BN;
  const bool use_product = !(alpha == 0.0 || K == 0);

  double acc[CF::FP][CF::GQ];
#pragma unroll
  for (int i = 0; i < CF::FP; ++i)
#pragma unroll
    for (int j = 0; j < CF::GQ; ++j) acc[i][j] = 0.0;

  // Position of acc[i][j] in C.  Lane 16 li + 4 lb4 + lj holds P index
  // p0 + 16 i + 4 lb4 + li and Q index q0 + 4 j + lj.
  const int li = lane >> 4, lb4 = (lane >> 2) & 3, lj = lane & 3;
  const int pofs = 4 * lb4 + li;
  auto c_row = [&](int i, int j) { return SW ? m0 + wm0 + 4 * j + lj : m0 + wm0 + 16 * i + pofs; };
  auto c_col = [&](int i, int j) { return SW ? n0 + wn0 + 16 * i + pofs : n0 + wn0 + 4 * j + lj; };

  // With beta != 0 the C tile is read up front so that its latency overlaps
  // the contraction instead of following it.
  constexpr bool CP = CF::CPRE;
  double cpre[CP ? CF::FP : 1][CP ? CF::GQ : 1];
  const bool prefetch_c = CP && use_product && beta != 0.0;
  if (prefetch_c) {
#pragma unroll
    for (int i = 0; i < CF::FP; ++i)
#pragma unroll
      for (int j = 0; j < CF::GQ; ++j) {
        const int row = c_row(i, j), col = c_col(i, j);
        const double x = C[(row < M ? row : M - 1) + (int64_t)(col < N ? col : N - 1) * ldc];
        cpre[CP ? i : 0][CP ? j : 0] = (row < M && col < N) ? x : 0.0;
      }
  }

  const bool pipe_ok = CF::PIPE >= 3 &&
                       (BG_PIPE_ANY_LD ? (aligned8(A_) && aligned8(B_))
                                       : (aligned16(A_) && aligned16(B_) && (lda % 2 == 0) &&
                                          (ldb % 2 == 0)));
  if constexpr (CF::PIPE >= 3) {
    if (use_product && pipe_ok) {
      using PS = PipeSmem<CF, TA, TB>;
      using TAs = typename PS::TAs;
      using TBs = typename PS::TBs;
      constexpr int NS = CF::PIPE;
      static_assert(NS <= 5 && 3 * PS::DPT <= 63, "wait counts must fit the vmcnt field");
      const int a_cext = TA ? K : M, a_sext = TA ? M : K;
      const int b_cext = TB ? N : K, b_sext = TB ? K : N;
      const int nk = (K + CF::BK - 1) / CF::BK;
      // The last k-step goes through registers when it is partial in k, or
      // when an MN-contiguous operand of odd extent is cut by this tile (its
      // last column must not be read past its end).
      const bool a_odd_edge = !TA && (M & 1) && (m0 + CF::BM > M);
      const bool b_odd_edge = TB && (N & 1) && (n0 + CF::BN > N);
      const bool last_tail = (K % CF::BK != 0) || a_odd_edge || b_odd_edge;
      auto issue = [&](int kt, int st) {
        const lptr la = lds + st * PS::STAGE, lb = la + TAs::ELEMS;
        const int k0 = kt * CF::BK;
        if (kt == nk - 1 && last_tail) {
          if (TA) tail_tile<TAs, CF::NT>(A, lda, k0, m0, a_cext, a_sext, la, tid);
          else    tail_tile<TAs, CF::NT>(A, lda, m0, k0, a_cext, a_sext, la, tid);
          if (TB) tail_tile<TBs, CF::NT>(B, ldb, n0, k0, b_cext, b_sext, lb, tid);
          else    tail_tile<TBs, CF::NT>(B, ldb, k0, n0, b_cext, b_sext, lb, tid);
        } else {
          if (TA) dma_tile<TAs, CF::NT>(A, lda, k0, m0, a_cext, a_sext, la, wave, lane);
          else    dma_tile<TAs, CF::NT>(A, lda, m0, k0, a_cext, a_sext, la, wave, lane);
          if (TB) dma_tile<TBs, CF::NT>(B, ldb, n0, k0, b_cext, b_sext, lb, wave, lane);
          else    dma_tile<TBs, CF::NT>(B, ldb, k0, n0, b_cext, b_sext, lb, wave, lane);
        }
      };
#pragma unroll
      for (int st = 0; st < NS - 1; ++st)
        if (st < nk) issue(st, st);
      const int p0 = SW ? wn0 : wm0, q0 = SW ? wm0 : wn0;
      // Step kt lives in stage kt mod NS.  Its loads are complete once at most
      // (steps issued after it) x DPT of this wave's loads remain; loads
      // return in order.  The barrier then publishes every wave's part, and
      // only after it is the stage read one step earlier refilled.  NPA of
      // the wave's FP slabs along P take part in the products (fewer on edge
      // tiles, see below); every wave issues the same loads and barriers.
      auto step = [&](int kt, auto stage_c, auto npa_c) {
        constexpr int st = decltype(stage_c)::value;
        constexpr int NPA = decltype(npa_c)::value;
        const int pending = min(NS - 2, nk - 1 - kt);
        asm volatile("" ::: "memory");
        if (pending <= 0) __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));
        else if (pending == 1) __builtin_amdgcn_s_waitcnt(waitcnt_imm(PS::DPT, 0));
        else if (pending == 2) __builtin_amdgcn_s_waitcnt(waitcnt_imm(2 * PS::DPT, 0));
        else __builtin_amdgcn_s_waitcnt(waitcnt_imm(3 * PS::DPT, 0));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // Wave priority raised from the barrier to the end of the step, and
        // the refill loads issued after the second fragment read: together
        // measured 1.4-4.5 % faster on 256^3, 512^3 and mixed-size batches.
        if constexpr (BG_PIPE_SETPRIO) __builtin_amdgcn_s_setprio(1);
        auto refill = [&]() {
          asm volatile("" ::: "memory");
          if (kt + NS - 1 < nk) issue(kt + NS - 1, (st + NS - 1) % NS);
          asm volatile("" ::: "memory");
        };
        if constexpr (NPA == 0 || !BG_PIPE_LATE_REFILL) refill();
        const lcptr la = lds + st * PS::STAGE, lb = la + TAs::ELEMS;
        const lcptr lp = SW ? lb : la;
        const lcptr lq = SW ? la : lb;
        if constexpr (NPA > 0) {
#pragma unroll
          for (int kk = 0; kk < CF::BK; kk += 16) {
            if (kt * CF::BK + kk >= K) break;  // whole 16-slices only, as on the other path
#pragma unroll
            for (int tp = 0; tp < 2; ++tp) {
              double fp[NPA][2], fq[CF::GQ][2];
              if constexpr (SW) {
                read_p_sw<TBs, NPA, !TB>(lp, p0, kk, tp, lane, fp);
                read_q_sw<TAs, CF::GQ, TA>(lq, q0, kk, tp, lane, fq);
              } else {
                read_p_sw<TAs, NPA, TA>(lp, p0, kk, tp, lane, fp);
                read_q_sw<TBs, CF::GQ, !TB>(lq, q0, kk, tp, lane, fq);
              }
              if constexpr (BG_PIPE_LATE_REFILL)
                if (kk == 0 && tp == 1) refill();
#pragma unroll
              for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < NPA; ++i)
#pragma unroll
                  for (int j = 0; j < CF::GQ; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f64_4x4x4f64(fp[i][u], fq[j][u], acc[i][j], 0, 0, 0);
            }
          }
        }
        if constexpr (BG_PIPE_SETPRIO) __builtin_amdgcn_s_setprio(0);
      };
      auto kloop = [&](auto npa_c) {
        for (int kt0 = 0; kt0 < nk; kt0 += NS) {
          step(kt0, std::integral_constant<int, 0>{}, npa_c);
          if (kt0 + 1 < nk) step(kt0 + 1, std::integral_constant<int, 1>{}, npa_c);
          if (kt0 + 2 < nk) step(kt0 + 2, std::integral_constant<int, 2>{}, npa_c);
          if constexpr (NS > 3)
            if (kt0 + 3 < nk) step(kt0 + 3, std::integral_constant<int, 3 % NS>{}, npa_c);
          if constexpr (NS > 4)
            if (kt0 + 4 < nk) step(kt0 + 4, std::integral_constant<int, 4 % NS>{}, npa_c);
        }
      };
      if constexpr (CF::SKIP >= 1) {
        // On edge tiles a wave whose region lies outside C does no products,
        // and a wave cut by the P edge computes only its slabs that reach into
        // C (16-wide granularity); the skipped sums only reach C elements
        // that are never stored.
        const int p_ext = SW ? N - n0 - wn0 : M - m0 - wm0;
        const int q_ext = SW ? M - m0 - wm0 : N - n0 - wn0;
        const int npa = (p_ext <= 0 || q_ext <= 0) ? 0 : min(CF::FP, (p_ext + 15) / 16);
        using std::integral_constant;
        constexpr int F = CF::FP;
        if (npa >= F) kloop(integral_constant<int, F>{});
        else if (npa == 0) kloop(integral_constant<int, 0>{});
        else if (npa == 1) kloop(integral_constant<int, 1>{});
        else if (npa == 2) kloop(integral_constant<int, (F > 2 ? 2 : F)>{});
        else if (npa == 3) kloop(integral_constant<int, (F > 3 ? 3 : F)>{});
        else kloop(integral_constant<int, F>{});
      } else {
        kloop(std::integral_constant<int, CF::FP>{});
      }
#ifndef BG_EPI_LDS
#define BG_EPI_LDS 1
#endif
      if constexpr (BG_EPI_LDS && CF::BM == 128 && CF::NT == 512 && SW) {
        // Interior tiles: the products go through LDS so that C is read and
        // written a whole column (1 KB) per instruction instead of 16
        // scattered 32-byte pieces per instruction.  Same arithmetic per
        // element as the epilogue below, so the results are bit-identical;
        // measured 2.3 % faster on the variable-size batch and up to 19 % on
        // short-k uniform batches (512 x 512 x 16).
#ifndef BG_EPI_XOR
#define BG_EPI_XOR 1
#endif
        // Column stride in LDS; with BG_EPI_XOR the columns are unpadded and
        // each column's 16-byte row pairs are XOR-swizzled by column, so the
        // products' writes (16 columns x 4 rows per instruction) hit distinct
        // banks in each half-wave, and the read-back of one column stays a
        // permutation of it (variable-size batch 0.9 % faster than padding
        // the columns by 4).
        constexpr int S = BG_EPI_XOR ? CF::BM : CF::BM + 4;
        constexpr int CPW = CF::BN / (CF::NT / 64);    // columns per wave
        static_assert(CF::BN * S <= PS::TOTAL, "C tile must fit the stages");
        auto epi_off = [](int c, int r) {  // LDS offset of tile element (row r, column c)
          if constexpr (BG_EPI_XOR)
            return c * S + 2 * ((r >> 1) ^ ((((c >> 2) + 4 * (c & 1)) & 7) << 1)) + (r & 1);
          else
            return c * S + r;
        };
        if (m0 + CF::BM <= M && n0 + CF::BN <= N && !CP) {
          const int wv = tid >> 6, ln = tid & 63;
          d2 cw[CPW];
          if (beta != 0.0) {
#pragma unroll
            for (int i = 0; i < CPW; ++i)
              cw[i] = ld_c((const AS_GLOBAL d2u*)(C + m0 + 2 * ln + (int64_t)(n0 + wv * CPW + i) * ldc));
          }
          __syncthreads();  // every wave is done reading the last stage
#pragma unroll
          for (int i = 0; i < CF::FP; ++i)
#pragma unroll
            for (int j = 0; j < CF::GQ; ++j)
              lds[epi_off(c_col(i, j) - n0, c_row(i, j) - m0)] = acc[i][j];
          __syncthreads();
#pragma unroll
          for (int i = 0; i < CPW; ++i) {
            const int cl = wv * CPW + i;
            const d2 a = *(const AS_LDS d2*)(lds + epi_off(cl, 2 * ln));
            d2 y;
            y.x = alpha * a.x;
            y.y = alpha * a.y;
            if (beta != 0.0) {
              y.x = y.x + beta * cw[i].x;
              y.y = y.y + beta * cw[i].y;
            }
            st_c((AS_GLOBAL d2u*)(C + m0 + 2 * ln + (int64_t)(n0 + cl) * ldc), (d2u)y);
          }
          return;
        }
#ifndef BG_EPI_LDS_EDGE
#define BG_EPI_LDS_EDGE 1
#endif
        if (BG_EPI_LDS_EDGE && !CP) {
          // Edge tile: the same column-wise form, each lane's row pair cut
          // at M (a lone last row is read and written alone) and columns
          // beyond N skipped; nothing outside C is read or written.
          // Measured 0.6-1.3 % faster on the variable-size batch.
          const int wv = tid >> 6, ln = tid & 63;
          const int r0 = m0 + 2 * ln;
          const bool one = r0 < M, pair = r0 + 1 < M;
          d2 cw[CPW];
          if (beta != 0.0) {
#pragma unroll
            for (int i = 0; i < CPW; ++i) {
              const int col = n0 + wv * CPW + i;
              cw[i].x = 0.0;
              cw[i].y = 0.0;
              if (col < N && one) {
                const gcptr pc = (gcptr)C + r0 + (int64_t)col * ldc;
                if (pair) cw[i] = *(const AS_GLOBAL d2u*)pc;
                else cw[i].x = pc[0];
              }
            }
          }
          __syncthreads();  // every wave is done reading the last stage
#pragma unroll
          for (int i = 0; i < CF::FP; ++i)
#pragma unroll
            for (int j = 0; j < CF::GQ; ++j)
              lds[epi_off(c_col(i, j) - n0, c_row(i, j) - m0)] = acc[i][j];
          __syncthreads();
#pragma unroll
          for (int i = 0; i < CPW; ++i) {
            const int cl = wv * CPW + i, col = n0 + cl;
            if (col < N && one) {
              const d2 a = *(const AS_LDS d2*)(lds + epi_off(cl, 2 * ln));
              d2 y;
              y.x = alpha * a.x;
              y.y = alpha * a.y;
              if (beta != 0.0) {
                y.x = y.x + beta * cw[i].x;
                y.y = y.y + beta * cw[i].y;
              }
              const gptr pc = C + r0 + (int64_t)col * ldc;
              if (pair) *(AS_GLOBAL d2u*)pc = y;
              else pc[0] = y.x;
            }
          }
          return;
        }
      }
    }
  }
  if (use_product && !(CF::PIPE >= 3 && pipe_ok)) {
    const lptr la0 = lds, lb0 = lds + CF::NSTAGE * SM::A_ELEMS;
    const int a_cext = TA ? K : M, a_sext = TA ? M : K;
    const int b_cext = TB ? N : K, b_sext = TB ? K : N;
    const bool a_vec = m0 + CF::BM <= M;
    const bool b_vec = n0 + CF::BN <= N;
    LA ra;
    LB rb;
    auto load = [&](int k0) {
      const bool kfull = k0 + CF::BK <= K;
      if (TA) ra.load(A, lda, k0, m0, a_cext, a_sext, a_vec && kfull, tid);
      else    ra.load(A, lda, m0, k0, a_cext, a_sext, a_vec && kfull, tid);
      if (TB) rb.load(B, ldb, n0, k0, b_cext, b_sext, b_vec && kfull, tid);
      else    rb.load(B, ldb, k0, n0, b_cext, b_sext, b_vec && kfull, tid);
    };
    const int nk = (K + CF::BK - 1) / CF::BK;
    load(0);
    ra.store(la0, tid);
    rb.store(lb0, tid);
    __syncthreads();
    const int p0 = SW ? wn0 : wm0, q0 = SW ? wm0 : wn0;
    // Valid extents of this wave's region along P and Q.  On edge tiles the
    // instructions whose 16 P indices or 4 Q indices all fall outside C are
    // skipped (wave-uniform tests); interior waves run without tests.
    const int p_ext = SW ? N - n0 - wn0 : M - m0 - wm0;
    const int q_ext = SW ? M - m0 - wm0 : N - n0 - wn0;
    const bool interior = p_ext >= CF::WP && q_ext >= CF::WQ;
    auto slice = [&](lcptr lp, lcptr lq, int kk, auto edge) {
      constexpr bool EDGE = decltype(edge)::value;
#pragma unroll
      for (int tp = 0; tp < 2; ++tp) {
        double fp[CF::FP][2], fq[CF::GQ][2];
        if constexpr (SW) {
          read_p<TBt, CF::FP, !TB>(lp, p0, kk, tp, lane, fp);
          read_q<TAt, CF::GQ, TA>(lq, q0, kk, tp, lane, fq);
        } else {
          read_p<TAt, CF::FP, TA>(lp, p0, kk, tp, lane, fp);
          read_q<TBt, CF::GQ, !TB>(lq, q0, kk, tp, lane, fq);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int i = 0; i < CF::FP; ++i)
#pragma unroll
            for (int j = 0; j < CF::GQ; ++j)
              if (!EDGE || (16 * i < p_ext && 4 * j < q_ext))
                acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(fp[i][u], fq[j][u], acc[i][j], 0, 0, 0);
      }
    };
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = CF::NSTAGE == 2 ? (kt & 1) : 0;
      if (kt + 1 < nk) load((kt + 1) * CF::BK);
      const lcptr la_cur = la0 + cur * SM::A_ELEMS, lb_cur = lb0 + cur * SM::B_ELEMS;
      const lcptr lp = SW ? lb_cur : la_cur;
      const lcptr lq = SW ? la_cur : lb_cur;
#pragma unroll
      for (int kk = 0; kk < CF::BK; kk += 16) {
        if (kt * CF::BK + kk >= K) break;  // whole 16-slices only, the same in every class
        if constexpr (CF::SKIP == 2) {
          if (interior) slice(lp, lq, kk, std::false_type{});
          else if (p_ext > 0 && q_ext > 0) slice(lp, lq, kk, std::true_type{});
        } else if constexpr (CF::SKIP == 1) {
          if (p_ext > 0 && q_ext > 0) slice(lp, lq, kk, std::false_type{});
        } else {
          slice(lp, lq, kk, std::false_type{});
        }
      }
      if (kt + 1 < nk) {
        if (CF::NSTAGE == 1) __syncthreads();  // every wave is done reading the stage
        const int nxt = CF::NSTAGE == 2 ? (cur ^ 1) : 0;
        ra.store(la0 + nxt * SM::A_ELEMS, tid);
        rb.store(lb0 + nxt * SM::B_ELEMS, tid);
      }
      __syncthreads();
    }
#ifndef BG_EPI_LDS_REG
#define BG_EPI_LDS_REG 1
#endif
    // The classes without the pipelined path take an LDS epilogue too (the
    // loop's last barrier has freed the stages): consecutive lanes handle
    // consecutive 16-byte row pairs of one column of C.
    constexpr int RS = CF::BM + 4;
    constexpr int RPAIRS = CF::BN * CF::BM / 2;
    if constexpr (BG_EPI_LDS_REG && CF::PIPE == 0 && !CF::CPRE && RPAIRS % CF::NT == 0 &&
                  CF::BN * RS <= TileSmem<CF, TA, TB>::TOTAL) {
      if (m0 + CF::BM <= M && n0 + CF::BN <= N) {
        constexpr int RPT = RPAIRS / CF::NT;
        d2 cw[RPT];
        if (beta != 0.0) {
#pragma unroll
          for (int it = 0; it < RPT; ++it) {
            const int u = it * CF::NT + tid, col = u / (CF::BM / 2), pr = u % (CF::BM / 2);
            cw[it] = ld_c((const AS_GLOBAL d2u*)(C + m0 + 2 * pr + (int64_t)(n0 + col) * ldc));
          }
        }
#pragma unroll
        for (int i = 0; i < CF::FP; ++i)
#pragma unroll
          for (int j = 0; j < CF::GQ; ++j)
            lds[(c_col(i, j) - n0) * RS + (c_row(i, j) - m0)] = acc[i][j];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < RPT; ++it) {
          const int u = it * CF::NT + tid, col = u / (CF::BM / 2), pr = u % (CF::BM / 2);
          const d2 a = *(const AS_LDS d2*)(lds + col * RS + 2 * pr);
          d2 y;
          y.x = alpha * a.x;
          y.y = alpha * a.y;
          if (beta != 0.0) {
            y.x = y.x + beta * cw[it].x;
            y.y = y.y + beta * cw[it].y;
          }
          st_c((AS_GLOBAL d2u*)(C + m0 + 2 * pr + (int64_t)(n0 + col) * ldc), (d2u)y);
        }
        return;
      }
#ifndef BG_EPI_LDS_REG_EDGE
#define BG_EPI_LDS_REG_EDGE 1
#endif
      if (BG_EPI_LDS_REG_EDGE && use_product) {
        // edge tile: row pairs cut at M, columns beyond N skipped, nothing
        // outside C read or written (measured 0.3-0.5 % faster on the
        // variable-size batches, whose small class is nearly all edge tiles)
        constexpr int RPT = RPAIRS / CF::NT;
        d2 cw[RPT];
        if (beta != 0.0) {
#pragma unroll
          for (int it = 0; it < RPT; ++it) {
            const int u = it * CF::NT + tid, col = n0 + u / (CF::BM / 2);
            const int r0 = m0 + 2 * (u % (CF::BM / 2));
            cw[it].x = 0.0;
            cw[it].y = 0.0;
            if (col < N && r0 < M) {
              const gcptr pc = (gcptr)C + r0 + (int64_t)col * ldc;
              if (r0 + 1 < M) cw[it] = *(const AS_GLOBAL d2u*)pc;
              else cw[it].x = pc[0];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < CF::FP; ++i)
#pragma unroll
          for (int j = 0; j < CF::GQ; ++j)
            lds[(c_col(i, j) - n0) * RS + (c_row(i, j) - m0)] = acc[i][j];
        __syncthreads();
#pragma unroll
        for (int it = 0; it < RPT; ++it) {
          const int u = it * CF::NT + tid, cl = u / (CF::BM / 2), pr = u % (CF::BM / 2);
          const int col = n0 + cl, r0 = m0 + 2 * pr;
          if (col < N && r0 < M) {
            const d2 a = *(const AS_LDS d2*)(lds + cl * RS + 2 * pr);
            d2 y;
            y.x = alpha * a.x;
            y.y = alpha * a.y;
            if (beta != 0.0) {
              y.x = y.x + beta * cw[it].x;
              y.y = y.y + beta * cw[it].y;
            }
            const gptr pc = C + r0 + (int64_t)col * ldc;
            if (r0 + 1 < M) *(AS_GLOBAL d2u*)pc = y;
            else pc[0] = y.x;
          }
        }
        return;
      }
    }
  }

  // Epilogue.  All C loads (beta != 0) are issued first, from clamped
  // in-bounds addresses, so they are in flight together; the stores are then
  // predicated on the C bounds (padding rows are never written).
  double cv[CF::FP][CF::GQ];
  const bool read_c = BG_EPI_BATCH && beta != 0.0 && !(use_product && prefetch_c);
  if (read_c) {
#pragma unroll
    for (int i = 0; i < CF::FP; ++i)
#pragma unroll
      for (int j = 0; j < CF::GQ; ++j) {
        const int row = c_row(i, j), col = c_col(i, j);
        cv[i][j] = C[(row < M ? row : M - 1) + (int64_t)(col < N ? col : N - 1) * ldc];
      }
  }
#pragma unroll
  for (int i = 0; i < CF::FP; ++i) {
#pragma unroll
    for (int j = 0; j < CF::GQ; ++j) {
      const int row = c_row(i, j), col = c_col(i, j);
      if (BG_EPI_BATCH) {
        const double c0v = (use_product && prefetch_c) ? cpre[CP ? i : 0][CP ? j : 0] : cv[i][j];
        double x;
        if (use_product) {
          x = alpha * acc[i][j];
          if (beta != 0.0) x = x + beta * c0v;
        } else {
          x = (beta == 0.0) ? 0.0 : beta * c0v;
        }
        // beta == 1 without a product leaves C untouched (never reached from
        // the uniform path, which returns early; a variable-size instance
        // with k == 0 and beta == 1 has no tiles)
        if (row < M && col < N && (use_product || beta != 1.0)) C[row + (int64_t)col * ldc] = x;
      } else {
        if (row >= M || col >= N) continue;
        const gptr p = C + row + (int64_t)col * ldc;
        if (use_product) {
          double x = alpha * acc[i][j];
          if (beta != 0.0) x = x + beta * (prefetch_c ? cpre[CP ? i : 0][CP ? j : 0] : *p);
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

// Waves per SIMD a tile kernel is compiled for (its register budget).  The
// 512-thread 'T','N' uniform kernel would take 132 VGPRs and run one
// workgroup per CU; held to 4 waves (128 VGPRs, the two workgroups its LDS
// allows) it still compiles without a spill, which the build checks, and
// runs 8 % faster.  The others fit 128 already ('N','N', 'T','T') or would
// spill ('N','T' and the variable-size 'T','N').
#ifndef BG_TN_WAVES
#define BG_TN_WAVES 4
#endif
template <class CF, bool TA, bool TB>
constexpr int uniform_min_waves() {
  return (CF::NT >= 512 && TA && !TB) ? BG_TN_WAVES : 1;
}

template <class CF, bool TA, bool TB>
__global__ __launch_bounds__(CF::NT, (uniform_min_waves<CF, TA, TB>())) void k_uniform(
    int M, int N, int K, double alpha, const double* const* __restrict__ Ap, int64_t lda,
    const double* const* __restrict__ Bp, int64_t ldb, double beta,
    double* const* __restrict__ Cp, int64_t ldc, int tiles_m, int tiles_per_inst,
    int64_t total_tiles, int64_t per_xcd) {
  __shared__ double lds[TileSmem<CF, TA, TB>::TOTAL];
  const int64_t bid = blockIdx.x;
  const int64_t id = (bid % NUM_XCD) * per_xcd + bid / NUM_XCD;
  if (id >= total_tiles) return;
  const int64_t inst = id / tiles_per_inst;
  const int t = (int)(id - inst * tiles_per_inst);
  const int tm = t % tiles_m, tn = t / tiles_m;
  gemm_tile<CF, TA, TB>(Ap[inst], lda, Bp[inst], ldb, Cp[inst], ldc, M, N, K, alpha, beta, tm,
                        tn, (lptr)lds);
}

// Persistent form for the pipelined class (1; off by default): one grid of
// resident workgroups that pop tiles from eight atomic queues, one per XCD
// range (as the variable-size executor does), each head on its own 4 KiB
// line of the handle's workspace, for batches with at least four k-steps per
// tile and four tiles per resident workgroup.  Measured 1 % faster than one
// workgroup per tile on 20,000 x 256^3, equal on 512^3 and up to 30 % faster
// on odd shapes (129 x 513 x 257), but it read 14 % (256^3) and 55 % (512^3)
// more from HBM than the algorithmic bytes, which one workgroup per tile
// matches exactly; a static deal of the tiles was slower.
#ifndef BG_UNIFORM_PERSIST
#define BG_UNIFORM_PERSIST 0
#endif
constexpr int UQ_STRIDE = 512;                   // int64 elements between heads
constexpr size_t UQ_BYTES = (size_t)NUM_XCD * UQ_STRIDE * 8;
// The persistent form is used when every workgroup gets this many tiles.
constexpr int64_t UQ_MIN_TILES_PER_WG = 4;

__global__ void k_uq_reset(unsigned long long* heads) {
  if (threadIdx.x < NUM_XCD) heads[threadIdx.x * UQ_STRIDE] = 0;
}

template <class CF, bool TA, bool TB>
__global__ __launch_bounds__(CF::NT, (uniform_min_waves<CF, TA, TB>())) void k_uniform_persist(
    int M, int N, int K, double alpha, const double* const* __restrict__ Ap, int64_t lda,
    const double* const* __restrict__ Bp, int64_t ldb, double beta,
    double* const* __restrict__ Cp, int64_t ldc, int tiles_m, int tiles_per_inst,
    int64_t total_tiles, unsigned long long* __restrict__ heads) {
  __shared__ double lds[TileSmem<CF, TA, TB>::TOTAL];
  __shared__ int64_t s_q;
  const int home = blockIdx.x % NUM_XCD;
  for (int step = 0; step < NUM_XCD; ++step) {
    const int x = (home + step) % NUM_XCD;
    const int64_t lo = total_tiles * x / NUM_XCD, hi = total_tiles * (x + 1) / NUM_XCD;
    for (;;) {
      if (threadIdx.x == 0) s_q = lo + (int64_t)atomicAdd(&heads[x * UQ_STRIDE], 1ull);
      __syncthreads();
      const int64_t id = s_q;
      __syncthreads();
      if (id >= hi) break;
      const int64_t inst = id / tiles_per_inst;
      const int t = (int)(id - inst * tiles_per_inst);
      gemm_tile<CF, TA, TB>(Ap[inst], lda, Bp[inst], ldb, Cp[inst], ldc, M, N, K, alpha, beta,
                            t % tiles_m, t / tiles_m, (lptr)lds);
      __syncthreads();  // LDS free for the next tile
    }
  }
}

template <class CF, bool TA, bool TB>
static hipError_t launch_uniform_t(const UniformArgs& a, hipStream_t s) {
  const int tiles_m = (a.m + CF::BM - 1) / CF::BM;
  const int tiles_n = (a.n + CF::BN - 1) / CF::BN;
  const int64_t tpi = (int64_t)tiles_m * tiles_n;
  const int64_t total = tpi * a.batch;
  if (tpi > INT32_MAX) return hipErrorInvalidValue;
  if (BG_UNIFORM_PERSIST && CF::PIPE >= 3 && a.num_cus > 0 && a.ws && a.ws_bytes >= UQ_BYTES) {
    auto kern = k_uniform_persist<CF, TA, TB>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, CF::NT, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const int64_t grid = (int64_t)a.num_cus * per_cu;
    if (total >= UQ_MIN_TILES_PER_WG * grid && a.k >= 4 * CF::BK) {
      unsigned long long* heads = (unsigned long long*)a.ws;
      hipLaunchKernelGGL(k_uq_reset, dim3(1), dim3(64), 0, s, heads);
      hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(CF::NT), 0, s, a.m, a.n, a.k, a.alpha,
                         a.A, a.lda, a.B, a.ldb, a.beta, a.C, a.ldc, tiles_m, (int)tpi, total,
                         heads);
      return hipGetLastError();
    }
  }
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

TileClass pick_uniform_class(int m, int n, int k, int batch, int num_cus, int force) {
  (void)k;
  if (force >= 0 && force < TC_COUNT) return (TileClass)force;
  const int mx = m > n ? m : n;
  if (mx <= 32) return TC_32;
  if (mx <= 64) return TC_64;
  // A batch too small to give every CU two 128 x 64 tiles is spread over
  // twice as many 64 x 64 tiles instead (a short batch is latency-bound:
  // more, shorter tiles finish sooner).
  const int64_t tiles128 = (int64_t)((m + Cfg128::BM - 1) / Cfg128::BM) *
                           ((n + Cfg128::BN - 1) / Cfg128::BN) * batch;
  if (tiles128 < 2 * (int64_t)num_cus) return TC_64;
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
// whole plan is made there.  Each instance is assigned one of three tile
// classes (128 x 64, 64 x 64, 32 x 32) by the padded work its C grid costs;
// each class gets its own tile queue, and a persistent kernel per class, in
// decreasing tile size, pops tiles from it:
//   1. k_vb_count: validate each instance (info), choose its class, count its
//      C tiles, and scan the counts of each class within blocks of 256;
//   2. k_vb_blocks: scan the block totals of each class (one workgroup),
//      reset the queues;
//   3. k_vb_finish: per-class exclusive prefix P_c[i] over instances;
//   4. k_vb_map: when it fits in the workspace, a map tile -> instance;
//   5. k_vb_exec (x3): a persistent grid per class; each workgroup pops tile
//      numbers from its class's atomic counters until the queue is empty.
// ---------------------------------------------------------------------------
#ifndef BG_CFGVB_L
#define BG_CFGVB_L 128, 64, 16, 32, 32, true
#endif
#ifndef BG_CFGVB_M
#define BG_CFGVB_M 64, 64, 16, 32, 32, true, 2, true
#endif
#ifndef BG_CFGVB_S
#define BG_CFGVB_S 32, 32, 16, 32, 32, false, 2, true
#endif
// relative cost per padded C element of the three classes, for the choice
#ifndef BG_VB_WEIGHTS
#define BG_VB_WEIGHTS 1.0f, 1.3f, 2.0f
#endif
using CfgVbL = Cfg<BG_CFGVB_L>;
using CfgVbM = Cfg<BG_CFGVB_M>;
using CfgVbS = Cfg<BG_CFGVB_S>;
constexpr int VB_NC = 3;
constexpr int PLAN_BLOCK = 256;
// Queue heads, one per (class, XCD), each on its own 4 KB line: every pop
// is a device-scope atomic, performed at the memory side, and heads sharing
// a line would serialise all pops of the device on one channel.
#ifndef BG_VB_HEAD_STRIDE
#define BG_VB_HEAD_STRIDE 512
#endif
constexpr int HEAD_STRIDE = BG_VB_HEAD_STRIDE;             // int64 elements
constexpr int HEAD_BASE = HEAD_STRIDE > VB_NC ? HEAD_STRIDE : VB_NC;
constexpr int VB_CTRL = HEAD_BASE + VB_NC * 8 * HEAD_STRIDE;  // totals, then the heads
__device__ __forceinline__ int64_t* vb_head(int64_t* ctrl, int cls, int x) {
  return ctrl + HEAD_BASE + (int64_t)(cls * 8 + x) * HEAD_STRIDE;
}

struct VbLayout {
  int64_t* prefix;   // [VB_NC][batch + 1]
  int64_t* bsum;     // [VB_NC][nblocks]
  int64_t* ctrl;     // [0..2] tiles per class, then the queue heads (vb_head)
  int* map;          // [map_cap]
  int64_t map_cap;
};

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t vbatched_workspace_bytes(int batch) {
  const size_t nb = ((size_t)batch + PLAN_BLOCK - 1) / PLAN_BLOCK;
  return align256(VB_NC * ((size_t)batch + 1) * 8) + align256(VB_NC * nb * 8) +
         align256(VB_CTRL * 8);
}

static VbLayout vb_layout(const VbWorkspace& ws, int batch) {
  VbLayout L;
  char* p = (char*)ws.base;
  const size_t nb = ((size_t)batch + PLAN_BLOCK - 1) / PLAN_BLOCK;
  L.prefix = (int64_t*)p; p += align256(VB_NC * ((size_t)batch + 1) * 8);
  L.bsum = (int64_t*)p; p += align256(VB_NC * nb * 8);
  L.ctrl = (int64_t*)p; p += align256(VB_CTRL * 8);
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

template <class CF>
__device__ __forceinline__ int64_t vb_tiles(int m, int n) {
  return (int64_t)((m + CF::BM - 1) / CF::BM) * ((n + CF::BN - 1) / CF::BN);
}

// Class with the least weighted padded C area; ties go to the larger tile.
__device__ __forceinline__ int vb_class(int m, int n, int64_t* tiles) {
  const float w[VB_NC] = {BG_VB_WEIGHTS};
  const int64_t t[VB_NC] = {vb_tiles<CfgVbL>(m, n), vb_tiles<CfgVbM>(m, n),
                            vb_tiles<CfgVbS>(m, n)};
  const float area[VB_NC] = {(float)(CfgVbL::BM * CfgVbL::BN), (float)(CfgVbM::BM * CfgVbM::BN),
                             (float)(CfgVbS::BM * CfgVbS::BN)};
  int best = 0;
  float cost = w[0] * area[0] * (float)t[0];
  for (int c = 1; c < VB_NC; ++c) {
    const float x = w[c] * area[c] * (float)t[c];
    if (x < cost) { cost = x; best = c; }
  }
  *tiles = t[best];
  return best;
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_count(
    bool ta, bool tb, const int* __restrict__ m, const int* __restrict__ n,
    const int* __restrict__ k, const int* __restrict__ lda, const int* __restrict__ ldb,
    const int* __restrict__ ldc, double alpha, double beta, int batch, int* __restrict__ info,
    int64_t* __restrict__ prefix, int64_t* __restrict__ bsum) {
  __shared__ int64_t sh[VB_NC][PLAN_BLOCK];
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  int64_t tiles = 0;
  int cls = 0;
  if (i < batch) {
    const int mi = m[i], ni = n[i], ki = k[i];
    const int st = vb_check(ta, tb, mi, ni, ki, lda[i], ldb[i], ldc[i]);
    if (info) info[i] = st;
    const bool noop = (alpha == 0.0 || ki == 0) && beta == 1.0;
    if (st == 0 && mi > 0 && ni > 0 && !noop) cls = vb_class(mi, ni, &tiles);
  }
  int64_t mine[VB_NC];
  for (int c = 0; c < VB_NC; ++c) {
    mine[c] = (c == cls) ? tiles : 0;
    sh[c][threadIdx.x] = mine[c];
  }
  __syncthreads();
  for (int off = 1; off < PLAN_BLOCK; off <<= 1) {  // inclusive scans (Hillis-Steele)
    int64_t x[VB_NC];
    for (int c = 0; c < VB_NC; ++c) x[c] = threadIdx.x >= off ? sh[c][threadIdx.x - off] : 0;
    __syncthreads();
    for (int c = 0; c < VB_NC; ++c) sh[c][threadIdx.x] += x[c];
    __syncthreads();
  }
  const int nb = gridDim.x;
  for (int c = 0; c < VB_NC; ++c) {
    if (i < batch) prefix[(int64_t)c * (batch + 1) + i] = sh[c][threadIdx.x] - mine[c];
    if (threadIdx.x == PLAN_BLOCK - 1) bsum[c * nb + blockIdx.x] = sh[c][PLAN_BLOCK - 1];
  }
}

__global__ __launch_bounds__(1024) void k_vb_blocks(int64_t* __restrict__ bsum, int nblocks,
                                                    int64_t* __restrict__ ctrl) {
  // exclusive scan of each class's block sums in place, 1024 per pass
  __shared__ int64_t sh[1024];
  __shared__ int64_t carry;
  for (int c = 0; c < VB_NC; ++c) {
    int64_t* b = bsum + (int64_t)c * nblocks;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 1024) {
      const int i = base + threadIdx.x;
      const int64_t x = i < nblocks ? b[i] : 0;
      sh[threadIdx.x] = x;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {
        const int64_t y = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
      }
      if (i < nblocks) b[i] = carry + sh[threadIdx.x] - x;
      __syncthreads();
      if (threadIdx.x == 1023) carry += sh[1023];
      __syncthreads();
    }
    if (threadIdx.x == 0) ctrl[c] = carry;                          // tiles of class c
    if (threadIdx.x < 8) *vb_head(ctrl, c, threadIdx.x) = 0;        // its per-XCD heads
    __syncthreads();
  }
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_finish(int batch, int64_t* __restrict__ prefix,
                                                          const int64_t* __restrict__ bsum,
                                                          const int64_t* __restrict__ ctrl) {
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  if (i >= batch) return;
  for (int c = 0; c < VB_NC; ++c) {
    int64_t* pc = prefix + (int64_t)c * (batch + 1);
    pc[i] += bsum[c * gridDim.x + blockIdx.x];
    if (i == batch - 1) pc[batch] = ctrl[c];
  }
}

// Writes the tile -> instance map (class c's tiles at offset sum_{c'<c} T_c')
// once all prefixes are final.
__global__ __launch_bounds__(PLAN_BLOCK) void k_vb_map(int batch, const int64_t* __restrict__ prefix,
                                                       const int64_t* __restrict__ ctrl,
                                                       int* __restrict__ map, int64_t map_cap) {
  int64_t total = 0;
  for (int c = 0; c < VB_NC; ++c) total += ctrl[c];
  if (total > map_cap) return;
  const int i = blockIdx.x * PLAN_BLOCK + threadIdx.x;
  if (i >= batch) return;
  int64_t moff = 0;
  for (int c = 0; c < VB_NC; ++c) {
    const int64_t* pc = prefix + (int64_t)c * (batch + 1);
    const int64_t lo = pc[i], hi = pc[i + 1];
    for (int64_t t = lo; t < hi; ++t) map[moff + t] = i;
    moff += ctrl[c];
  }
}

// Instance owning tile q of a class: the last i with P[i] <= q < P[i + 1].
__device__ __forceinline__ int vb_find(const int64_t* __restrict__ prefix, int batch, int64_t q) {
  int lo = 0, hi = batch;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

// The tiles of a class are split into eight equal ranges, one per XCD
// (workgroups reach the XCDs round-robin by id), so that the tiles of an
// instance run on one XCD and share its L2 for the A and B panels.  A
// workgroup pops from its own XCD's range first, then steals from the others
// in turn; every counter is only ever incremented, so each tile is taken
// exactly once and every workgroup leaves after one pass over the eight.
template <class CF, bool TA, bool TB>
__global__ __launch_bounds__(CF::NT) void k_vb_exec(
    const int* __restrict__ m, const int* __restrict__ n, const int* __restrict__ k, double alpha,
    const double* const* __restrict__ Ap, const int* __restrict__ lda,
    const double* const* __restrict__ Bp, const int* __restrict__ ldb, double beta,
    double* const* __restrict__ Cp, const int* __restrict__ ldc, int batch, int cls,
    const int64_t* __restrict__ prefix_all, int64_t* __restrict__ ctrl, const int* __restrict__ map,
    int64_t map_cap) {
  __shared__ double lds[TileSmem<CF, TA, TB>::TOTAL];
  __shared__ int64_t s_q;
  const int64_t* prefix = prefix_all + (int64_t)cls * (batch + 1);
  const int64_t total = ctrl[cls];
  if (total == 0) return;   // no tile of this class (uniform across the workgroup)
  int64_t all = 0, moff = 0;
  for (int c = 0; c < VB_NC; ++c) {
    all += ctrl[c];
    if (c < cls) moff += ctrl[c];
  }
  const bool use_map = all <= map_cap;

  const int home = blockIdx.x % NUM_XCD;
  for (int step = 0; step < NUM_XCD; ++step) {
    const int x = (home + step) % NUM_XCD;
    const int64_t lo = total * x / NUM_XCD, hi = total * (x + 1) / NUM_XCD;
    for (;;) {
      if (threadIdx.x == 0)
        s_q = lo + (int64_t)atomicAdd((unsigned long long*)vb_head(ctrl, cls, x), 1ull);
      __syncthreads();
      const int64_t q = s_q;
      __syncthreads();
      if (q >= hi) break;
      const int i = use_map ? map[moff + q] : vb_find(prefix, batch, q);
      const int mi = m[i], ni = n[i], ki = k[i];
      const int tiles_m = (mi + CF::BM - 1) / CF::BM;
      const int t = (int)(q - prefix[i]);
      gemm_tile<CF, TA, TB>(Ap[i], lda[i], Bp[i], ldb[i], Cp[i], ldc[i], mi, ni, ki, alpha, beta,
                            t % tiles_m, t / tiles_m, (lptr)lds);
      __syncthreads();  // LDS free for the next tile
    }
  }
}

template <class CF, bool TA, bool TB>
static hipError_t launch_vb_exec(const VbatchedArgs& a, const VbLayout& L, int cls, int num_cus,
                                 hipStream_t s) {
  auto kern = k_vb_exec<CF, TA, TB>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, CF::NT, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  hipLaunchKernelGGL(kern, dim3(num_cus * per_cu), dim3(CF::NT), 0, s, a.m, a.n, a.k, a.alpha,
                     a.A, a.lda, a.B, a.ldb, a.beta, a.C, a.ldc, a.batch, cls, L.prefix, L.ctrl,
                     L.map, L.map_cap);
  return hipGetLastError();
}

template <class CF>
static hipError_t launch_vb_exec_t(const VbatchedArgs& a, const VbLayout& L, int cls, int num_cus,
                                   hipStream_t s) {
  if (!a.ta && !a.tb) return launch_vb_exec<CF, false, false>(a, L, cls, num_cus, s);
  if (!a.ta && a.tb) return launch_vb_exec<CF, false, true>(a, L, cls, num_cus, s);
  if (a.ta && !a.tb) return launch_vb_exec<CF, true, false>(a, L, cls, num_cus, s);
  return launch_vb_exec<CF, true, true>(a, L, cls, num_cus, s);
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
  if ((e = launch_vb_exec_t<CfgVbL>(a, L, 0, num_cus, s)) != hipSuccess) return e;
  if ((e = launch_vb_exec_t<CfgVbM>(a, L, 1, num_cus, s)) != hipSuccess) return e;
  return launch_vb_exec_t<CfgVbS>(a, L, 2, num_cus, s);
}

}  // namespace bg
