// Internal declarations shared by the C-ABI layer (bgemm_api.cpp) and the
// kernel launchers (bgemm_kernels.hip).  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bg {

// Tile shapes.  A "size class" is one tile configuration of the MFMA tile
// kernel: C tile BM x BN per workgroup, contraction step BK per LDS stage,
// each wave computing a WM x WN sub-tile with 4x4x4 FP64 MFMAs (the exact
// shapes come from the BG_CFG* macros, i.e. the tune cache).
enum TileClass : int {
  TC_32 = 0,     // 32 x 32 tile         (tiny matrices)
  TC_64 = 1,     // 64 x 64 tile         (small matrices, short batches)
  TC_128 = 2,    // 128 x 64 tile        (large matrices)
  TC_COUNT = 3
};

struct TileShape { int bm, bn, bk, threads; };
TileShape tile_shape(TileClass c);

// Picks the tile class for a uniform batch of `batch` instances on a device
// of `num_cus` compute units; `force` >= 0 overrides.
TileClass pick_uniform_class(int m, int n, int k, int batch, int num_cus, int force);

struct UniformArgs {
  bool ta, tb;
  int m, n, k;
  double alpha, beta;
  const double* const* A; int64_t lda;
  const double* const* B; int64_t ldb;
  double* const* C; int64_t ldc;
  int batch;
  int num_cus = 0;   // compute units of the device (sizes persistent grids)
  void* ws = nullptr;         // handle workspace (queue heads of the persistent form)
  size_t ws_bytes = 0;
};

// Launches the uniform batched GEMM (product path; alpha != 0, k > 0).
hipError_t launch_uniform(const UniformArgs& a, TileClass cls, hipStream_t s);

// Reduced / emulated precision modes of the uniform batch (NN operands only):
// mode 1 binary32, 2 bfloat16, 3 emulated binary64 with `slices` (1..8)
// bfloat16 digit slices.  hipErrorInvalidValue for grids beyond int32.
hipError_t launch_uniform_lowp(const UniformArgs& a, int mode, int slices, hipStream_t s);
// Emulated binary64 on int8 digit slices (NN, k <= 8192): per group of
// instances, row / column exponents into the workspace (m + n ints per
// instance), then the product.  hipErrorInvalidValue when the workspace holds
// no instance or slices is outside 1..8.
hipError_t launch_emu8(const UniformArgs& a, int slices, void* ws, size_t ws_bytes, hipStream_t s);

// Launches C_i <- beta * C_i (beta != 1) for every instance, used when the
// product term vanishes (alpha == 0 or k == 0).
hipError_t launch_scale(double beta, double* const* C, int64_t ldc, int m, int n, int batch,
                        hipStream_t s);

struct VbatchedArgs {
  bool ta, tb;
  const int *m, *n, *k;
  double alpha, beta;
  const double* const* A; const int* lda;
  const double* const* B; const int* ldb;
  double* const* C; const int* ldc;
  int batch;
  int* info;  // nullable
};

// Host-side argument rules of the variable-size call (0 when valid, else the
// reference-BLAS argument number) and the argument pack built from them.
int vbatched_host_args(char transa, char transb, const int* d_m, const int* d_n, const int* d_k,
                       const void* dA, const int* d_lda, const void* dB, const int* d_ldb,
                       const void* dC, const int* d_ldc, int batch);
VbatchedArgs vbatched_args(char transa, char transb, const int* d_m, const int* d_n,
                           const int* d_k, double alpha, const double* const* dA,
                           const int* d_lda, const double* const* dB, const int* d_ldb,
                           double beta, double* const* dC, const int* d_ldc, int batch,
                           int* d_info);

// Workspace layout used by the vbatched planner and executor.
struct VbWorkspace {
  void* base;
  size_t bytes;
};

// Bytes of workspace the planner needs for `batch` instances, excluding the
// optional tile map (which uses whatever remains).
size_t vbatched_workspace_bytes(int batch);

// Plans (validate, count tiles, prefix sums, tile map) and executes the
// variable-size batch with a persistent kernel; all on stream `s`.
hipError_t launch_vbatched(const VbatchedArgs& a, const VbWorkspace& ws, int num_cus,
                           hipStream_t s);

// Complex uniform batch (interleaved binary64 pairs; ld in complex elements;
// op codes 0 N, 1 T, 2 C; alpha and beta point to host (re, im) pairs).
struct ZUniformArgs {
  int ta, tb;
  int m, n, k;
  const double* alpha;
  const double* beta;
  const double* const* A; int64_t lda;
  const double* const* B; int64_t ldb;
  double* const* C; int64_t ldc;
  int batch;
};
hipError_t launch_zgemm(const ZUniformArgs& a, hipStream_t s);
// C_i <- beta C_i for complex C (beta == 0 writes exact zeros, C not read).
hipError_t launch_zscale(const double* beta, double* const* C, int64_t ldc, int m, int n,
                         int batch, hipStream_t s);

// Two-spin gates on batches of 2^S-amplitude states (in place).
hipError_t launch_gate2(int S, const int* sites, const double* const* U, double* const* psi,
                        int batch, int* info, hipStream_t s);

// Request loop: one generated factor (column-major n x n at `out`; factor j of
// `client`, values scaled by `scale`).
struct FillJob {
  double* out;
  long long j;
  int n;
  int client;
  double scale;
};

// Generates the factors of njobs jobs (device array) in one launch; max_n is
// the largest n among them.
hipError_t launch_fill_factors(const FillJob* d_jobs, int njobs, int max_n,
                               unsigned long long seed, hipStream_t s);
// One factor, the same generator (host-side job).
hipError_t launch_fill_one(double* out, int n, int client, long long j, double scale,
                           unsigned long long seed, hipStream_t s);
// Annealing sweeps: factor t of a sweep for each job reads the client's
// product count at the start of the sweep from j0 (device) and uses
// j = j0[client] + t; k_advance adds `chain` to every j0 entry.
struct SweepJob {
  double* out;
  int n;
  int client;
  double scale;
};
hipError_t launch_fill_sweep(const SweepJob* d_jobs, int njobs, int max_n, const long long* d_j0,
                             int t, unsigned long long seed, hipStream_t s);
hipError_t launch_advance(long long* d_j0, int n, int chain, hipStream_t s);
// out <- identity (n x n, column-major, ld = n).
hipError_t launch_identity(double* out, int n, hipStream_t s);

}  // namespace bg
