// Native GEMM kernels for op(A) = A^T, op(B) = B^T (its own translation unit so the
// layout combinations compile in parallel).
#include "gemm_launch.h"

namespace mg {

int gemm_tiles_tt(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha,
                  const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                  int64_t ldc, hipStream_t s) {
  return gemm_tiles<true, true>(dtype, cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

}  // namespace mg
