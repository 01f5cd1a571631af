/*
 * CPU oracle for batched dense GEMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never calls it,
 * and the two share no code: no headers, helpers, tables or constants.
 *
 * What it computes (the paper, Section II, Eq. 1): for every instance i,
 *     C_i <- alpha * op(A_i) * op(B_i) + beta * C_i
 * with op(X) = X for 'N'/'n' and X^T for 'T'/'t'/'C'/'c' (real data, so the
 * conjugate transpose is the transpose).  op(A_i) is m x k, op(B_i) is k x n,
 * C_i is m x n.  Every matrix is column-major: element (r, c) of a matrix with
 * leading dimension ld sits at offset r + c * ld.  Instances are independent
 * of each other (Section III: the Monte Carlo procedures exchange no data).
 *
 * The arithmetic is the plain definition written out, in a fixed order:
 *   for each column j of C: acc[r] = sum over p = 0, 1, ..., k-1 (ascending)
 *   of opA(r, p) * opB(p, j), one rounded multiply and one rounded add per
 *   term (the build passes -ffp-contract=off, so no fused multiply-add).
 *   Then, the BLAS conventions for the scalars (the paper names BLAS in its
 *   introduction and is silent on the special cases):
 *     beta == 0                 : C = alpha*acc (C is never read; alpha == 0
 *                                 or k == 0 gives exactly 0)
 *     alpha == 0 or k == 0      : C = beta*C   (A and B are never read; beta
 *                                 == 1 leaves C untouched)
 *     otherwise                 : C = fl(alpha*acc) + fl(beta*C)
 *   Rows of the ld padding (r >= m) are never read or written.
 *
 * Argument rules (reference-BLAS ordering of DGEMM's argument numbers):
 *   1 transa, 2 transb, 3 m, 4 n, 5 k, 8 lda, 10 ldb, 13 ldc.
 * lda >= max(1, rows of A as stored) where that is m for 'N' and k for 'T';
 * ldb >= max(1, k for 'N', n for 'T'); ldc >= max(1, m).
 *
 * Parallelism: OpenMP over instances only; one instance is computed by one
 * thread, so results do not depend on the thread count.
 */
#include <stdlib.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 0 = no transpose, 1 = transpose, -1 = not a valid character */
static int trans_code(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

static int imax1(int a) { return a > 1 ? a : 1; }

/* Returns 0 when the arguments are valid, else -(argument number). */
int oracle_check_args(char transa, char transb, int m, int n, int k,
                      int lda, int ldb, int ldc)
{
    int ta = trans_code(transa), tb = trans_code(transb);
    if (ta < 0) return -1;
    if (tb < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (k < 0) return -5;
    if (lda < imax1(ta ? k : m)) return -8;
    if (ldb < imax1(tb ? n : k)) return -10;
    if (ldc < imax1(m)) return -13;
    return 0;
}

/* One instance.  Returns 0, or -(argument number) without touching C. */
int oracle_dgemm(char transa, char transb, int m, int n, int k, double alpha,
                 const double *A, int lda, const double *B, int ldb,
                 double beta, double *C, int ldc)
{
    int info = oracle_check_args(transa, transb, m, n, k, lda, ldb, ldc);
    if (info != 0) return info;
    if (m == 0 || n == 0) return 0;

    int ta = trans_code(transa), tb = trans_code(transb);
    int64_t slda = lda, sldb = ldb, sldc = ldc;
    int use_product = !(alpha == 0.0 || k == 0);

    double *acc = (double *)malloc(sizeof(double) * (size_t)m);
    if (!acc) return -100;

    for (int j = 0; j < n; ++j) {
        double *cj = C + (int64_t)j * sldc;
        if (use_product) {
            for (int r = 0; r < m; ++r) acc[r] = 0.0;
            for (int p = 0; p < k; ++p) {
                /* opB(p, j): B(p, j) for 'N', B(j, p) for 'T' */
                double b = tb ? B[(int64_t)j + (int64_t)p * sldb]
                              : B[(int64_t)p + (int64_t)j * sldb];
                for (int r = 0; r < m; ++r) {
                    /* opA(r, p): A(r, p) for 'N', A(p, r) for 'T' */
                    double a = ta ? A[(int64_t)p + (int64_t)r * slda]
                                  : A[(int64_t)r + (int64_t)p * slda];
                    double t = a * b;
                    acc[r] = acc[r] + t;
                }
            }
        }
        for (int r = 0; r < m; ++r) {
            if (beta == 0.0) {
                cj[r] = use_product ? alpha * acc[r] : 0.0;
            } else if (!use_product) {
                if (beta != 1.0) cj[r] = beta * cj[r];
            } else {
                double x = alpha * acc[r];
                double y = beta * cj[r];
                cj[r] = x + y;
            }
        }
    }
    free(acc);
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Uniform sizes, host pointer arrays.  Returns 0, or -(argument number) for
 * an invalid shared argument (14 = batch), or -100 on allocation failure. */
int oracle_dgemm_batched(char transa, char transb, int m, int n, int k,
                         double alpha, const double *const *A, int lda,
                         const double *const *B, int ldb, double beta,
                         double *const *C, int ldc, int batch, int nthreads)
{
    int info = oracle_check_args(transa, transb, m, n, k, lda, ldb, ldc);
    if (info != 0) return info;
    if (batch < 0) return -14;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int i = 0; i < batch; ++i) {
        int r = oracle_dgemm(transa, transb, m, n, k, alpha, A[i], lda, B[i],
                             ldb, beta, C[i], ldc);
        if (r != 0) failed = 1;
    }
    return failed ? -100 : 0;
}

/* Per-instance sizes, host arrays.  info[i] (if info is not NULL) receives 0
 * for a computed instance or -(argument number) for an instance whose sizes
 * break the argument rules; such an instance's C is left untouched.  The
 * return value is -1/-2 for a bad trans character, -14 for batch < 0, -100
 * on allocation failure, else 0. */
int oracle_dgemm_vbatched(char transa, char transb, const int *m, const int *n,
                          const int *k, double alpha, const double *const *A,
                          const int *lda, const double *const *B,
                          const int *ldb, double beta, double *const *C,
                          const int *ldc, int batch, int *info, int nthreads)
{
    if (trans_code(transa) < 0) return -1;
    if (trans_code(transb) < 0) return -2;
    if (batch < 0) return -14;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int i = 0; i < batch; ++i) {
        int r = oracle_dgemm(transa, transb, m[i], n[i], k[i], alpha, A[i],
                             lda[i], B[i], ldb[i], beta, C[i], ldc[i]);
        if (r == -100) failed = 1;
        if (info) info[i] = (r == -100) ? 0 : r;
    }
    return failed ? -100 : 0;
}

/* ------------------------------------------------------------------------
 * Complex instances (the paper's matrices are complex, Section II, Eq. 1).
 * Elements are interleaved (real, imaginary) binary64 pairs; element (r, c)
 * of a matrix with leading dimension ld (in complex elements) has its real
 * part at 2 (r + c ld) and its imaginary part right after.  op(X) = X for
 * 'N', X^T for 'T', the conjugate transpose X^H for 'C'.  alpha and beta are
 * (real, imaginary) pairs.
 *
 * Arithmetic, in the plain order: the complex product is the real product of
 * the embedded operands, so each output part is a real dot product of length
 * 2k whose terms are taken for p = 0, 1, ..., k-1 in turn:
 *     acc_re = acc_re + a_re * b_re;  acc_re = acc_re + (-a_im) * b_im;
 *     acc_im = acc_im + a_im * b_re;  acc_im = acc_im + a_re * b_im;
 * (a = opA(r, p), b = opB(p, j); each product and each add rounded).  Then
 * x = alpha acc and y = beta C as (p_re q_re - p_im q_im, p_re q_im + p_im q_re)
 * with every product and the add / subtract rounded, and C = x + y part by
 * part.  Scalar rules (BLAS): beta == 0 never reads C; alpha == 0 or k == 0
 * never reads A or B and gives C = beta C (beta == 1 leaves C untouched).
 * Argument numbers as for the real call (1 transa, 2 transb, 3 m, 4 n, 5 k,
 * 8 lda, 10 ldb, 13 ldc); 'C' counts as a transpose for the ld rules.
 * ------------------------------------------------------------------------ */
static int ztrans_code(char t)
{
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't') return 1;
    if (t == 'C' || t == 'c') return 2;
    return -1;
}

int oracle_zgemm(char transa, char transb, int m, int n, int k, const double *alpha,
                 const double *A, int lda, const double *B, int ldb,
                 const double *beta, double *C, int ldc)
{
    int info = oracle_check_args(transa, transb, m, n, k, lda, ldb, ldc);
    if (info != 0) return info;
    if (m == 0 || n == 0) return 0;
    int ta = ztrans_code(transa), tb = ztrans_code(transb);
    int64_t slda = lda, sldb = ldb, sldc = ldc;
    const double ar_ = alpha[0], ai_ = alpha[1], br_ = beta[0], bi_ = beta[1];
    int alpha_zero = (ar_ == 0.0 && ai_ == 0.0);
    int beta_zero = (br_ == 0.0 && bi_ == 0.0);
    int beta_one = (br_ == 1.0 && bi_ == 0.0);
    int use_product = !(alpha_zero || k == 0);

    double *acc = (double *)malloc(sizeof(double) * 2 * (size_t)m);
    if (!acc) return -100;
    for (int j = 0; j < n; ++j) {
        double *cj = C + 2 * (int64_t)j * sldc;
        if (use_product) {
            for (int r = 0; r < 2 * m; ++r) acc[r] = 0.0;
            for (int p = 0; p < k; p++) {
                const double *bp = tb ? B + 2 * ((int64_t)j + (int64_t)p * sldb)
                                      : B + 2 * ((int64_t)p + (int64_t)j * sldb);
                double bre = bp[0], bim = tb == 2 ? -bp[1] : bp[1];
                for (int r = 0; r < m; ++r) {
                    const double *ap = ta ? A + 2 * ((int64_t)p + (int64_t)r * slda)
                                          : A + 2 * ((int64_t)r + (int64_t)p * slda);
                    double are = ap[0], aim = ta == 2 ? -ap[1] : ap[1];
                    double t;
                    t = are * bre;    acc[2 * r] = acc[2 * r] + t;
                    t = (-aim) * bim; acc[2 * r] = acc[2 * r] + t;
                    t = aim * bre;    acc[2 * r + 1] = acc[2 * r + 1] + t;
                    t = are * bim;    acc[2 * r + 1] = acc[2 * r + 1] + t;
                }
            }
        }
        for (int r = 0; r < m; ++r) {
            double *c = cj + 2 * r;
            if (!use_product) {
                if (beta_zero) { c[0] = 0.0; c[1] = 0.0; }
                else if (!beta_one) {
                    double yr = br_ * c[0] - bi_ * c[1];
                    double yi = br_ * c[1] + bi_ * c[0];
                    c[0] = yr; c[1] = yi;
                }
                continue;
            }
            double xr = ar_ * acc[2 * r] - ai_ * acc[2 * r + 1];
            double xi = ar_ * acc[2 * r + 1] + ai_ * acc[2 * r];
            if (beta_zero) { c[0] = xr; c[1] = xi; continue; }
            double yr = br_ * c[0] - bi_ * c[1];
            double yi = br_ * c[1] + bi_ * c[0];
            c[0] = xr + yr;
            c[1] = xi + yi;
        }
    }
    free(acc);
    return 0;
}

int oracle_zgemm_batched(char transa, char transb, int m, int n, int k,
                         const double *alpha, const double *const *A, int lda,
                         const double *const *B, int ldb, const double *beta,
                         double *const *C, int ldc, int batch, int nthreads)
{
    int info = oracle_check_args(transa, transb, m, n, k, lda, ldb, ldc);
    if (info != 0) return info;
    if (ztrans_code(transa) < 0) return -1;
    if (ztrans_code(transb) < 0) return -2;
    if (batch < 0) return -14;
    int failed = 0;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int i = 0; i < batch; ++i) {
        int r = oracle_zgemm(transa, transb, m, n, k, alpha, A[i], lda, B[i], ldb,
                             beta, C[i], ldc);
        if (r != 0) failed = 1;
    }
    return failed ? -100 : 0;
}
