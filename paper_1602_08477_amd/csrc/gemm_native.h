// Host-side entry points of the native FP64/FP32 tiled GEMM.
#pragma once

#include "common.h"

namespace mg {

// True if 16-byte vector access is safe: base aligned to esz*vec bytes and
// the row pitch a multiple of vec elements.
bool vec_aligned(const void *p, int64_t ld, int64_t esz, int vec);

int num_tile_cfgs();
int tile_cfg_info(int dtype, int cfg, int *bm, int *bn, int *bk, int *threads);
int pick_tile_cfg(int dtype, int64_t m, int64_t n, int64_t k);

// Enqueues C <- alpha*A*B + beta*C with work division `cfg` (arguments
// already validated).
int gemm_native(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                hipStream_t s);

// Same with op(A) = A^T (A stored k x m) when ta, op(B) = B^T (B stored
// n x k) when tb.
int gemm_native_op(int dtype, int cfg, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                   double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                   double beta, void *C, int64_t ldc, hipStream_t s);

// The tiled kernels of one layout combination (one translation unit each);
// m, n, k >= 1 and alpha != 0.
#define MG_GEMM_TILES_DECL(name)                                                               \
  int name(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,   \
           int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,         \
           hipStream_t s)
MG_GEMM_TILES_DECL(gemm_tiles_nn);
MG_GEMM_TILES_DECL(gemm_tiles_tn);
MG_GEMM_TILES_DECL(gemm_tiles_nt);
MG_GEMM_TILES_DECL(gemm_tiles_tt);
#undef MG_GEMM_TILES_DECL

}  // namespace mg
