/*
 * CPU oracle for the generalised matrix-matrix multiply C <- alpha*A*B + beta*C
 * (the DGEMM problem of Section 4.2, "Performance", of the Alpaka paper), and
 * for DAXPY y <- alpha*x + y (Section 4.1), at the end of this file.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the bench's CPU-baseline
 * leg do.  It shares no code, header or constant with the HIP library.
 *
 * Definition computed (plain, per output element, no blocking or reordering):
 *     C[i][j] <- alpha * sum_{p<k} A[i][p] * B[p][j] + beta * C[i][j]
 * Matrices are row-major with a row pitch ("leading dimension") in elements,
 * the paper's 1-D buffers with aligned rows.
 *
 * Accuracy: the dot product is accumulated with the compensated algorithm
 * Dot2 of Ogita, Rump and Oishi ("Accurate sum and dot product", SIAM J. Sci.
 * Comput. 26(6), 2005): every product is split exactly into value + error
 * with an FMA (TwoProduct) and every addition into value + error with Knuth's
 * TwoSum; the error terms are summed separately.  The result is as accurate as
 * if the dot product had been formed in twice the working precision.  The
 * final alpha*s + beta*c is formed in double-double and rounded once.
 *
 * The loop order is i (rows, OpenMP), then p (k), then j, keeping one (s, c)
 * pair per output column of the current row; for a fixed (i, j) the terms are
 * still added in increasing p, exactly as the sum is written.
 *
 * Special cases follow the BLAS convention (the paper does not state them):
 * beta == 0 means C is not read (so NaN/Inf in C do not propagate);
 * alpha == 0 or k == 0 means A and B are not read and C <- beta*C.
 *
 * Must be compiled with -ffp-contract=off and without -ffast-math: TwoSum and
 * TwoProduct rely on every + and * being rounded exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Knuth's TwoSum: a + b = *s + *e exactly. */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* TwoProduct with an FMA: a * b = *p + *e exactly (no underflow). */
static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* alpha*(hi + lo) + beta*c, evaluated in double-double, rounded once. */
static inline double finish(double alpha, double s, double cerr, double beta,
                            const double *cij)
{
    double hi, lo, p1, e1, p2 = 0.0, e2 = 0.0, t, e3;
    two_sum(s, cerr, &hi, &lo);
    two_prod(alpha, hi, &p1, &e1);
    e1 += alpha * lo;
    if (beta != 0.0)
        two_prod(beta, *cij, &p2, &e2);
    two_sum(p1, p2, &t, &e3);
    return t + (e1 + (e2 + e3));
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Returns 0 on success, -1 on invalid arguments, -2 if scratch allocation fails. */
int oracle_dgemm(int64_t m, int64_t n, int64_t k, double alpha,
                 const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc)
{
    if (m < 0 || n < 0 || k < 0)
        return -1;
    if (m == 0 || n == 0)
        return 0;
    if (ldc < n || C == NULL)
        return -1;

    if (k == 0 || alpha == 0.0) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                C[i * ldc + j] = (beta == 0.0) ? 0.0 : beta * C[i * ldc + j];
        return 0;
    }
    if (A == NULL || B == NULL || lda < k || ldb < n)
        return -1;

    int failed = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc((size_t)n * sizeof(double));
        double *c = (double *)malloc((size_t)n * sizeof(double));
        if (s == NULL || c == NULL) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < m; ++i) {
                for (int64_t j = 0; j < n; ++j) {
                    s[j] = 0.0;
                    c[j] = 0.0;
                }
                const double *arow = A + i * lda;
                for (int64_t p = 0; p < k; ++p) {
                    const double a = arow[p];
                    const double *brow = B + p * ldb;
                    for (int64_t j = 0; j < n; ++j) {
                        double prod, perr, sum, serr;
                        two_prod(a, brow[j], &prod, &perr);
                        two_sum(s[j], prod, &sum, &serr);
                        s[j] = sum;
                        c[j] += serr + perr;
                    }
                }
                double *crow = C + i * ldc;
                for (int64_t j = 0; j < n; ++j)
                    crow[j] = finish(alpha, s[j], c[j], beta, crow + j);
            }
        }
        free(s);
        free(c);
    }
    return failed ? -2 : 0;
}

/*
 * DAXPY, the vector operation of the paper's conceptual comparison (Section
 * 4.1): y <- alpha*x + y, element i of x at x[i*incx] and of y at y[i*incy].
 * Each element is the exact value alpha*x[i] + y[i] rounded once to the
 * nearest double (C99 fma, correctly rounded), the most accurate result a
 * double can hold.  BLAS quick return: n == 0 or alpha == 0 leaves y as it is
 * and reads nothing.  Returns 0, or -1 for negative n or increments below 1.
 */
int oracle_daxpy(int64_t n, double alpha, const double *x, int64_t incx, double *y,
                 int64_t incy)
{
    if (n < 0 || incx < 1 || incy < 1)
        return -1;
    if (n == 0 || alpha == 0.0)
        return 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        y[i * incy] = fma(alpha, x[i * incx], y[i * incy]);
    return 0;
}
