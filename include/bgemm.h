/*
 * bgemm -- batched FP64 GEMM for AMD Instinct MI355X (CDNA4, gfx950).
 *
 * The operation is the paper's Eq. 1 (Section II): for i = 1..N,
 *     C_i <- alpha * op(A_i) * op(B_i) + beta * C_i
 * over a very large batch of small, independent instances, real FP64.
 * op(X) = X for transX = 'N'/'n' and X^T for 'T'/'t'/'C'/'c' (real data, so
 * the conjugate transpose is the transpose).  op(A_i) is m x k, op(B_i) is
 * k x n, C_i is m x n.
 *
 * Layout.  Every matrix is column-major: element (r, c) of a matrix with
 * leading dimension ld is at offset r + c * ld (doubles).  A with 'N' is
 * stored m x k (lda >= max(1, m)); with 'T' it is stored k x m
 * (lda >= max(1, k)).  B with 'N' is stored k x n (ldb >= max(1, k)); with 'T'
 * n x k (ldb >= max(1, n)).  ldc >= max(1, m).  Rows r >= rows of a column
 * (the ld padding) are never written, and their values never reach a stored
 * result.  They may be read: when a column length is odd, a 16-byte load at
 * the end of a column (other than the last column of the matrix) can take
 * the element after it with it -- the first padding element, or the next
 * column's first element when ld equals the column length; that element
 * only enters products for C rows or columns outside C, which are
 * discarded.  The padding must therefore be readable memory (it is, by
 * ld >= rows), but its contents (NaN included) never matter.  Operands need
 * 8-byte alignment.
 *
 * Memory and ownership.  Matrices, the pointer arrays dA/dB/dC (one device
 * pointer per instance), the per-instance size arrays of the variable-size
 * call and d_info are DEVICE memory owned by the caller; the library never
 * frees or retains them.  alpha and beta are host values.  The handle owns
 * only its workspace, allocated by bg_create / bg_set_workspace (the
 * variable-size planner's buffers; in builds with the persistent uniform form
 * its first 32 KiB also hold that form's tile queues); no compute entry point
 * allocates.
 *
 * Semantics of the scalars (reference BLAS; the paper is silent):
 *   beta == 0            C is not read (NaN in C does not propagate);
 *   alpha == 0 or k == 0 A and B are not read; C <- beta * C, exactly 0 when
 *                        beta == 0, untouched (bit-identical) when beta == 1;
 *   m == 0 or n == 0     nothing happens.
 *
 * Aliasing.  C_i may not overlap any C_j (j != i), A_j or B_j.  A_i and B_i
 * may alias each other (Gram products).  Results do not depend on the order
 * of the instances in the pointer arrays or on what else is in the batch:
 * each instance's summation order is fixed by its own sizes.
 *
 * Synchronisation.  Calls are asynchronous on the handle's stream: SUCCESS
 * means the work was enqueued.  A device fault surfaces as BG_STATUS_DEVICE_ERROR
 * from a later call or from the caller's stream synchronisation.
 *
 * Threads.  A handle is not thread-safe; use one handle per host thread.
 */
#ifndef BGEMM_H
#define BGEMM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BG_STATUS_SUCCESS = 0,
  BG_STATUS_INVALID_VALUE = 1,   /* an argument breaks the rules below */
  BG_STATUS_NOT_SUPPORTED = 2,   /* valid but outside this build (e.g. sizes beyond int32 grids) */
  BG_STATUS_DEVICE_ERROR = 3,    /* a HIP call failed */
  BG_STATUS_ALLOC_FAILED = 4,    /* workspace allocation failed */
  BG_STATUS_INVALID_HANDLE = 5,  /* NULL or destroyed handle */
  BG_STATUS_WORKSPACE_TOO_SMALL = 6 /* variable-size batch larger than the workspace plans for */
} bg_status_t;

typedef struct bg_handle* bg_handle_t;

/* Library version as 10000 * major + 100 * minor + patch. */
int bg_version(void);

/* Static string naming a status code. */
const char* bg_status_string(bg_status_t s);

/* Creates a handle bound to the current HIP device, with the default stream
 * and a workspace of BG_DEFAULT_WORKSPACE_BYTES (the environment variable
 * BG_WORKSPACE_MB overrides the size).  *h is set only on success. */
#define BG_DEFAULT_WORKSPACE_BYTES (64u << 20)
bg_status_t bg_create(bg_handle_t* h);

/* Frees the handle's workspace.  Work already enqueued must have finished
 * (the call synchronises the handle's stream first). */
bg_status_t bg_destroy(bg_handle_t h);

/* Sets the stream (a hipStream_t; NULL = the default stream) that later
 * calls enqueue on. */
bg_status_t bg_set_stream(bg_handle_t h, void* stream);
bg_status_t bg_get_stream(bg_handle_t h, void** stream);

/* Replaces the workspace with one of `bytes` bytes (synchronises the stream).
 * The variable-size call needs bg_workspace_bytes_needed(batch) bytes of
 * planning space (about 24 * (batch + 1) bytes of prefix sums plus 96 KiB of
 * queue heads, each on its own 4 KiB line) plus, for its fastest schedule,
 * 4 bytes per C tile. */
bg_status_t bg_set_workspace(bg_handle_t h, unsigned long long bytes);
unsigned long long bg_workspace_bytes_needed(int batch);

/* Argument number (reference-BLAS DGEMM numbering: 1 transa, 2 transb, 3 m,
 * 4 n, 5 k, 7 A, 8 lda, 9 B, 10 ldb, 12 C, 13 ldc, 14 batch) of the first
 * invalid argument of the handle's last call, 0 if that call was valid. */
int bg_last_invalid_arg(bg_handle_t h);

/* Host-only check of a uniform batched call's arguments, in the order above;
 * touches no device.  Returns 0 when valid, else the argument number. */
int bg_check_batched_args(char transa, char transb, int m, int n, int k,
                          const void* dA, int lda, const void* dB, int ldb,
                          const void* dC, int ldc, int batch);

/* Uniform sizes (the paper's fixed-size batch, Section II): every instance is
 * m x n x k with the same leading dimensions.  Quick returns, with no launch:
 * batch == 0, m == 0, n == 0, and (alpha == 0 or k == 0) with beta == 1.
 * Returns BG_STATUS_INVALID_VALUE (and records the argument number) for
 * a bad trans character, m/n/k < 0, lda/ldb/ldc below their minimum,
 * batch < 0, or a NULL pointer array when batch > 0 and the array is read. */
bg_status_t bg_dgemm_batched(bg_handle_t h, char transa, char transb,
                             int m, int n, int k, double alpha,
                             const double* const* dA, int lda,
                             const double* const* dB, int ldb, double beta,
                             double* const* dC, int ldc, int batch);

/* Variable sizes (the paper's variable-size batch, Section II): instance i
 * has sizes d_m[i], d_n[i], d_k[i] and leading dimensions d_lda[i], d_ldb[i],
 * d_ldc[i] (all device int arrays of length batch).  The sizes are checked on
 * the device: an instance that breaks the rules gets d_info[i] = -(argument
 * number: 3 m, 4 n, 5 k, 8 lda, 10 ldb, 13 ldc) and its C is left untouched;
 * a valid one gets d_info[i] = 0.  d_info may be NULL.  All instances go into
 * one persistent launch that pops C tiles from a device-side queue; planning
 * is done on the device, so the host never reads the sizes.  Host-side
 * errors: a bad trans character, batch < 0, NULL arrays when batch > 0, or
 * BG_STATUS_WORKSPACE_TOO_SMALL. */
bg_status_t bg_dgemm_vbatched(bg_handle_t h, char transa, char transb,
                              const int* d_m, const int* d_n, const int* d_k,
                              double alpha,
                              const double* const* dA, const int* d_lda,
                              const double* const* dB, const int* d_ldb,
                              double beta,
                              double* const* dC, const int* d_ldc,
                              int batch, int* d_info);

/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * variable-size call of bg_dgemm_vbatched without a handle.  Arguments,
 * layout, device-side size checks, d_info and results are those of
 * bg_dgemm_vbatched (bit-identical results); the work is enqueued on
 * `stream` (a hipStream_t, NULL = default stream) of the CURRENT device.
 * Nothing is allocated: the planner's buffers live in one static device
 * array of BG_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends (its address is looked up on the first call on
 * that device).  Every call on a GPU reuses that GPU's array and overwrites
 * it, so calls that may overlap on one GPU (different streams, concurrent
 * host threads with no ordering between their streams) race and must not be
 * issued; calls ordered on one stream are safe.  Batches whose planning
 * buffers do not fit the array (batch > bg_noalloc_max_batch(), about 690,000)
 * return BG_STATUS_WORKSPACE_TOO_SMALL with nothing enqueued; very large tile
 * counts are served without the optional tile map (same results).  Host
 * argument errors return BG_STATUS_INVALID_VALUE and, when bad_arg is not
 * NULL, set *bad_arg to the argument number of bg_dgemm_vbatched's rules (0
 * when valid). */
#define BG_NOALLOC_SCRATCH_BYTES (16u << 20)
int bg_noalloc_max_batch(void);
bg_status_t bg_dgemm_vbatched_noalloc(void* stream, char transa, char transb,
                                      const int* d_m, const int* d_n, const int* d_k,
                                      double alpha,
                                      const double* const* dA, const int* d_lda,
                                      const double* const* dB, const int* d_ldb,
                                      double beta,
                                      double* const* dC, const int* d_ldc,
                                      int batch, int* d_info, int* bad_arg);

/* Arithmetic of bg_gemm_batched_mode.  Inputs and outputs stay binary64; only
 * the arithmetic inside the product changes:
 *   BG_MODE_FP64  the binary64 path of bg_dgemm_batched (slices ignored);
 *   BG_MODE_FP32  A and B rounded to binary32 (nearest even), products summed
 *                 in binary32 on the matrix cores;
 *   BG_MODE_BF16  A and B rounded to binary32 and then to bfloat16 (nearest
 *                 even at each step), products summed in binary32;
 *   BG_MODE_EMU   binary64 emulated with `slices` (1..8) bfloat16 digit slices
 *                 per operand: per 32-wide chunk of k each row of A and column
 *                 of B is scaled by a power of two into (-1, 1) and cut into
 *                 8-bit signed digits; the digit products up to the
 *                 (slices + 1)-th diagonal are summed exactly in binary32 and
 *                 recombined in binary64 in a fixed order, so every result is
 *                 reproducible bit for bit.  The error falls by about 2^-8 per
 *                 added slice; 7 slices reach the binary64 path's accuracy on
 *                 well-scaled data.
 *   BG_MODE_EMU_I8 binary64 emulated with `slices` (1..8) int8 digit slices
 *                 per operand (Ozaki et al., Numer. Algorithms 59, 2012): each
 *                 row of A and column of B is scaled over all of k by a power
 *                 of two, rounded to an integer of 8 * slices - 1 bits and
 *                 cut into signed base-256 digits; the digit products up to
 *                 the (slices + 1)-th diagonal are summed exactly in int32 on
 *                 the int8 matrix cores and recombined in binary64 in a fixed
 *                 order (bit-reproducible).  Needs k <= 8192 (else
 *                 NOT_SUPPORTED) and (m + n) * 4 bytes of the handle's
 *                 workspace per instance for at least one instance (else
 *                 ALLOC_FAILED); larger batches run in groups that fit.
 *                 Finite inputs only.  The error is bounded by about
 *                 slices * k * 2^(2 - 8 slices) * 2^(e_i + f_j) per entry (e_i,
 *                 f_j the exponents of row i's and column j's largest
 *                 magnitudes); 7 slices stay within 1e-14 relative on data
 *                 spread over 2^+-20, 8 match the binary64 path.
 *   BG_MODE_EMU_F32 the digits, diagonals and recombination of BG_MODE_EMU
 *                 with the digit products summed on the binary32 matrix
 *                 cores (digits converted exactly to binary32; every partial
 *                 sum is an integer below 2^24), so its results are
 *                 bit-identical to BG_MODE_EMU with the same `slices`.
 * The paper computes in binary64 only (Section II); these modes are an
 * extension for callers that trade accuracy for matrix-core throughput. */
typedef enum {
  BG_MODE_FP64 = 0,
  BG_MODE_FP32 = 1,
  BG_MODE_BF16 = 2,
  BG_MODE_EMU = 3,
  BG_MODE_EMU_I8 = 4,
  BG_MODE_EMU_F32 = 5
} bg_mode_t;

/* Uniform batch as bg_dgemm_batched, computed in `mode`.  Arguments, layout,
 * ownership, quick returns and the alpha/beta rules are those of
 * bg_dgemm_batched (alpha == 0 or k == 0 gives C <- beta * C in binary64 for
 * every mode).  The reduced modes take non-transposed operands only
 * (transa == transb == 'N'); a transposed operand with such a mode returns
 * BG_STATUS_NOT_SUPPORTED.  A bad mode records argument number 101, a slice
 * count outside 1..8 for BG_MODE_EMU, BG_MODE_EMU_I8 or BG_MODE_EMU_F32
 * records 102 (both
 * INVALID_VALUE). */
bg_status_t bg_gemm_batched_mode(bg_handle_t h, int mode, int slices, char transa, char transb,
                                 int m, int n, int k, double alpha,
                                 const double* const* dA, int lda,
                                 const double* const* dB, int ldb, double beta,
                                 double* const* dC, int ldc, int batch);

/* Complex uniform batch (the paper's matrices are complex, Section II, Eq. 1):
 * C_i <- alpha op(A_i) op(B_i) + beta C_i with op(X) = X ('N'), X^T ('T') or
 * the conjugate transpose X^H ('C').  Elements are interleaved (real,
 * imaginary) binary64 pairs (the layout of C99 double complex); leading
 * dimensions count complex elements; alpha and beta point to host (real,
 * imaginary) pairs.  Argument rules, numbering, quick returns and scalar
 * rules follow bg_dgemm_batched (alpha == 0 means both parts zero; beta == 1
 * means 1 + 0i); a NULL alpha or beta records argument 6 or 11.  Operands
 * need 8-byte alignment. */
bg_status_t bg_zgemm_batched(bg_handle_t h, char transa, char transb,
                             int m, int n, int k, const double* alpha,
                             const double* const* dA, int lda,
                             const double* const* dB, int ldb, const double* beta,
                             double* const* dC, int ldc, int batch);

/* Two-spin gates on a batch of S-spin states (the paper's Monte Carlo step
 * applies a local unitary to a random pair of neighbouring spins, Section
 * III, Alg. 1; the paper gives no gate model, so any 4 x 4 complex matrix
 * is accepted).  State i (dPsi[i], 2^S interleaved binary64 complex
 * amplitudes, 16-byte alignment recommended) is updated in place: amplitude
 * x has spin j in bit j of x, and for site s = d_site[i] the gate
 * dU[i] (4 x 4 complex, column-major: element (q, q') at 2 (q + 4 q'))
 * maps every quadruple of amplitudes that differ only in bits s and s + 1
 * (local index q = b_s + 2 b_{s+1}) to U times itself.  d_site, dU, dPsi and
 * d_info (nullable; 0 done, -3 for a site outside 0..S-2, that state left
 * untouched) are device arrays of length batch.  Host errors: S outside
 * 2..40 (argument 2), NULL arrays when batch > 0 (3, 4, 5), batch < 0 (6). */
bg_status_t bg_zgate2_batched(bg_handle_t h, int S, const int* d_site,
                              const double* const* dU, double* const* dPsi, int batch,
                              int* d_info);

/* Overrides the size class chosen for uniform batches (-1 = automatic;
 * 0 = 32x32 tiles, 1 = 64x64, 2 = 128x128).  For tuning and tests. */
bg_status_t bg_set_uniform_class(bg_handle_t h, int cls);

#ifdef __cplusplus
}
#endif
#endif /* BGEMM_H */
