/*
 * Drives the CPU oracle (oracle/mg_oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Every operand sits in a heap block of exactly
 * the size its extent and pitch need, so a read or write one element past a
 * row or past the matrix lands in a redzone.  Small-integer entries make
 * every sum exact, so the results are checked bit for bit against a plain
 * integer triple loop.  Special cases: beta == 0 with NaN in C (C not read),
 * alpha == 0 and k == 0 with NULL A and B (A and B not read).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_dgemm(int64_t m, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta, double *C, int64_t ldc);
int oracle_daxpy(int64_t n, double alpha, const double *x, int64_t incx, double *y,
                 int64_t incy);
void oracle_set_threads(int n);

static int failures = 0;

static double *block(int64_t rows, int64_t cols, int64_t ld) {
  const int64_t count = rows > 0 && cols > 0 ? (rows - 1) * ld + cols : 1;
  double *p = (double *)malloc((size_t)count * sizeof(double));
  if (!p) abort();
  return p;
}

static double small_int(int64_t i, int64_t j, int salt) {
  return (double)(((i * 7 + j * 13 + salt * 5) % 17) - 8);
}

static void check_gemm(int64_t m, int64_t n, int64_t k, int64_t pad, double alpha, double beta) {
  const int64_t lda = k + pad, ldb = n + pad, ldc = n + pad;
  double *A = (k > 0 && alpha != 0.0) ? block(m, k, lda) : NULL;
  double *B = (k > 0 && alpha != 0.0) ? block(k, n, ldb) : NULL;
  double *C = block(m, n, ldc);
  double *want = block(m, n, n);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t p = 0; p < k && A; ++p) A[i * lda + p] = small_int(i, p, 1);
  for (int64_t p = 0; p < k && B; ++p)
    for (int64_t j = 0; j < n; ++j) B[p * ldb + j] = small_int(p, j, 2);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      C[i * ldc + j] = beta == 0.0 ? NAN : small_int(i, j, 3);
      long long s = 0;
      for (int64_t p = 0; p < k && A; ++p)
        s += (long long)small_int(i, p, 1) * (long long)small_int(p, j, 2);
      want[i * n + j] = alpha * (double)s + (beta == 0.0 ? 0.0 : beta * small_int(i, j, 3));
    }
  const int rc = oracle_dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  if (rc != 0) {
    fprintf(stderr, "oracle_dgemm rc=%d for m=%lld n=%lld k=%lld\n", rc, (long long)m,
            (long long)n, (long long)k);
    ++failures;
  }
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j)
      if (C[i * ldc + j] != want[i * n + j]) {
        fprintf(stderr, "mismatch m=%lld n=%lld k=%lld at (%lld,%lld): %g vs %g\n",
                (long long)m, (long long)n, (long long)k, (long long)i, (long long)j,
                C[i * ldc + j], want[i * n + j]);
        ++failures;
        i = m;
        break;
      }
  free(A);
  free(B);
  free(C);
  free(want);
}

static void check_axpy(int64_t n, int64_t incx, int64_t incy) {
  const int64_t nx = n > 0 ? (n - 1) * incx + 1 : 1, ny = n > 0 ? (n - 1) * incy + 1 : 1;
  double *x = (double *)malloc((size_t)nx * sizeof(double));
  double *y = (double *)malloc((size_t)ny * sizeof(double));
  if (!x || !y) abort();
  for (int64_t i = 0; i < nx; ++i) x[i] = small_int(i, 0, 4);
  for (int64_t i = 0; i < ny; ++i) y[i] = small_int(i, 1, 5);
  if (oracle_daxpy(n, 1.5, x, incx, y, incy) != 0) ++failures;
  for (int64_t i = 0; i < n; ++i)
    if (y[i * incy] != 1.5 * small_int(i * incx, 0, 4) + small_int(i * incy, 1, 5)) {
      fprintf(stderr, "daxpy mismatch n=%lld at %lld\n", (long long)n, (long long)i);
      ++failures;
      break;
    }
  free(x);
  free(y);
}

int main(void) {
  for (int th = 1; th <= 4; th *= 4) {
    oracle_set_threads(th);
    for (int64_t m = 0; m <= 9; ++m)
      for (int64_t n = 0; n <= 9; ++n)
        for (int64_t k = 0; k <= 9; k += 3) {
          check_gemm(m, n, k, 0, 1.5, 0.5);
          check_gemm(m, n, k, 3, 1.0, 0.0);
        }
    check_gemm(37, 70, 129, 1, 1.5, 0.5);
    check_gemm(65, 33, 17, 0, 0.0, 2.0);
    check_gemm(40, 41, 0, 2, 1.0, 0.25);
  }
  for (int64_t n = 0; n <= 40; n += 7)
    for (int64_t incx = 1; incx <= 3; ++incx)
      for (int64_t incy = 1; incy <= 3; ++incy) check_axpy(n, incx, incy);
  if (oracle_dgemm(-1, 1, 1, 1.0, NULL, 1, NULL, 1, 0.0, NULL, 1) == 0) ++failures;
  if (oracle_daxpy(4, 1.0, NULL, 0, NULL, 1) == 0) ++failures;
  printf("oracle under sanitizers: %d failures\n", failures);
  return failures != 0;
}
