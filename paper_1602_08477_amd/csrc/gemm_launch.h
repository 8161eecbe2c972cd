// Native FP64 / FP32 GEMM kernels and their launchers, templated on the
// operand layouts: C <- alpha*op(A)*op(B) + beta*C with op(X) = X or X^T
// (one workgroup per macro-tile of C, Section 4.2.2 tiling).  Each layout
// combination is instantiated by its own translation unit.
#pragma once

#include "gemm_dma.h"
#include "gemm_native.h"
#include "gemm_tile.h"

namespace mg {

namespace {

constexpr int kGroupM = 8;  // tile-rows walked together by the raster

template <typename T, int BM, int BN, bool VEC_OK, int WGM, int WGN, int BKM, bool TA, bool TB>
__global__ __launch_bounds__((TileShape<T, BM, BN, WGM, WGN, BKM>::THREADS)) void gemm_native_kernel(
    GemmArgs<T> g, int tiles_m, int tiles_n) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *smem = reinterpret_cast<T *>(lds_raw);
  int tm, tn;
  const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  grouped_tile(t, tiles_m, tiles_n, kGroupM, tm, tn);
  gemm_tile<T, BM, BN, VEC_OK, WGM, WGN, BKM, TA, TB>(g, tm * BM, tn * BN, smem);
}

template <typename T, int BM, int BN, int WGM, int WGN, int NS, bool TA, bool TB, int KS = 1>
__global__ __launch_bounds__((DmaShape<T, BM, BN, WGM, WGN, NS, KS>::THREADS),
                             (DmaShape<T, BM, BN, WGM, WGN, NS, KS>::MINW)) void gemm_dma_kernel(
    GemmArgs<T> g, int tiles_m, int tiles_n) {
  extern __shared__ __align__(16) unsigned char lds[];
  int tm, tn;
  const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  grouped_tile(t, tiles_m, tiles_n, kGroupM, tm, tn);
  gemm_dma_tile<T, BM, BN, WGM, WGN, NS, TA, TB, KS>(g, tm * BM, tn * BN, lds);
}

// The textbook mapping without the paper's hierarchy below the thread: one
// output per lane, no shared memory, the k loop reading A and B straight
// from global memory (the naive triple loop of Section 4.2's portability
// experiment).  Lanes of a 16 x 16 workgroup take consecutive columns, so
// B and C accesses coalesce and A values are shared by a row of lanes.
// The sum runs in increasing k with one FMA per term.
constexpr int kNaiveDim = 16;

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(kNaiveDim *kNaiveDim) void gemm_naive_kernel(GemmArgs<T> g) {
  const int j = blockIdx.x * kNaiveDim + threadIdx.x;
  const int i = blockIdx.y * kNaiveDim + threadIdx.y;
  if (i >= g.m || j >= g.n) return;
  T s = T(0);
  for (int p = 0; p < g.k; ++p) {
    const T a = TA ? g.A[(int64_t)p * g.lda + i] : g.A[(int64_t)i * g.lda + p];
    const T b = TB ? g.B[(int64_t)j * g.ldb + p] : g.B[(int64_t)p * g.ldb + j];
    s = fma(a, b, s);
  }
  T *c = g.C + (int64_t)i * g.ldc + j;
  *c = g.beta != T(0) ? fma(g.alpha, s, g.beta * *c) : g.alpha * s;
}

template <typename T, bool TA, bool TB>
int launch_naive(const GemmArgs<T> &g, hipStream_t s) {
  const int64_t bx = (g.n + kNaiveDim - 1) / kNaiveDim, by = (g.m + kNaiveDim - 1) / kNaiveDim;
  if (by > 65535 || bx * by * kNaiveDim * kNaiveDim > (int64_t)UINT32_MAX) {
    set_error("naive work division: %d x %d outputs exceed one dispatch", g.m, g.n);
    return MG_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL((gemm_naive_kernel<T, TA, TB>), dim3((unsigned)bx, (unsigned)by),
                     dim3(kNaiveDim, kNaiveDim), 0, s, g);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

// Raises a kernel's dynamic LDS limit to what its ring needs; called through
// a function-local static, so once per template instance and thread-safe.
template <typename K>
hipError_t set_max_lds(K kern, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int BM, int BN, bool VEC_OK, int WGM, int WGN, int BKM, bool TA, bool TB>
int launch_one(const GemmArgs<T> &g, hipStream_t s) {
  typedef TileShape<T, BM, BN, WGM, WGN, BKM, TA, TB> S;
  const int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  if (tiles * S::THREADS > (int64_t)UINT32_MAX) {  // 32-bit work-item count per dispatch
    set_error("too many tiles (%lld) for one dispatch", (long long)tiles);
    return MG_ERR_INVALID_ARG;
  }
  auto kern = gemm_native_kernel<T, BM, BN, VEC_OK, WGM, WGN, BKM, TA, TB>;
  static const hipError_t attr = set_max_lds(kern, S::LDS_BYTES);  // once per instance
  MG_HIP_TRY(attr);
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(S::THREADS), S::LDS_BYTES, s, g, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <typename T, int BM, int BN, int WGM, int WGN, int NS, bool TA, bool TB, int KS = 1>
int launch_dma(const GemmArgs<T> &g, hipStream_t s) {
  typedef DmaShape<T, BM, BN, WGM, WGN, NS, KS> S;
  const int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  if (tiles * S::THREADS > (int64_t)UINT32_MAX) {  // 32-bit work-item count per dispatch
    set_error("too many tiles (%lld) for one dispatch", (long long)tiles);
    return MG_ERR_INVALID_ARG;
  }
  auto kern = gemm_dma_kernel<T, BM, BN, WGM, WGN, NS, TA, TB, KS>;
  static const hipError_t attr = set_max_lds(kern, S::LDS_BYTES);  // once per instance
  MG_HIP_TRY(attr);
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(S::THREADS), S::LDS_BYTES, s, g, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

// Work divisions 0-13 stage A and B through registers; 14-24 load them
// straight into an LDS ring (16-byte aligned operands only: otherwise a
// register-staged division of the same macro-tile runs); 25 is the naive
// one-output-per-lane mapping; 26-29 are direct-load rings whose wavefronts
// form two k groups (twice the wavefronts per output block).  The host's table
// of shapes (kCfgs in gemm_native.hip) lists the same divisions in order.
template <typename T, bool V, bool TA, bool TB>
int launch_cfg(int cfg, const GemmArgs<T> &g, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_one<T, 128, 128, V, 2, 2, 1, TA, TB>(g, s);
    case 1: return launch_one<T, 128, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 2: return launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 3: return launch_one<T, 64, 32, V, 2, 2, 1, TA, TB>(g, s);
    case 4: return launch_one<T, 32, 32, V, 2, 2, 1, TA, TB>(g, s);
    case 5: return launch_one<T, 128, 128, V, 4, 2, 1, TA, TB>(g, s);
    case 6: return launch_one<T, 128, 128, V, 2, 4, 1, TA, TB>(g, s);
    case 7: return launch_one<T, 64, 64, V, 2, 2, 2, TA, TB>(g, s);
    case 8: return launch_one<T, 128, 64, V, 4, 2, 1, TA, TB>(g, s);
    case 9: return launch_one<T, 128, 64, V, 2, 2, 2, TA, TB>(g, s);
    case 10: return launch_one<T, 256, 128, V, 4, 2, 1, TA, TB>(g, s);
    case 11: return launch_one<T, 128, 256, V, 2, 4, 1, TA, TB>(g, s);
    case 12: return launch_one<T, 256, 128, V, 4, 4, 1, TA, TB>(g, s);
    case 13: return launch_one<T, 128, 128, V, 4, 2, 2, TA, TB>(g, s);
    case 14:
      return V ? launch_dma<T, 64, 64, 2, 2, 4, TA, TB>(g, s)
               : launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 15:
      return V ? launch_dma<T, 64, 32, 2, 2, 4, TA, TB>(g, s)
               : launch_one<T, 64, 32, V, 2, 2, 1, TA, TB>(g, s);
    case 16:
      return V ? launch_dma<T, 128, 64, 2, 2, 4, TA, TB>(g, s)
               : launch_one<T, 128, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 17:
      return V ? launch_dma<T, 128, 128, 2, 4, 3, TA, TB>(g, s)
               : launch_one<T, 128, 128, V, 4, 2, 2, TA, TB>(g, s);
    case 18:
      return V ? launch_dma<T, 256, 128, 4, 4, 3, TA, TB>(g, s)
               : launch_one<T, 256, 128, V, 4, 4, 1, TA, TB>(g, s);
    case 19:
      return V ? launch_dma<T, 32, 32, 2, 2, 4, TA, TB>(g, s)
               : launch_one<T, 32, 32, V, 2, 2, 1, TA, TB>(g, s);
    case 20:
      return V ? launch_dma<T, 64, 64, 4, 2, 4, TA, TB>(g, s)
               : launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 21:
      return V ? launch_dma<T, 128, 128, 2, 4, 2, TA, TB>(g, s)
               : launch_one<T, 128, 128, V, 4, 2, 2, TA, TB>(g, s);
    case 22:
      return V ? launch_dma<T, 128, 128, 2, 2, 2, TA, TB>(g, s)
               : launch_one<T, 128, 128, V, 4, 2, 2, TA, TB>(g, s);
    case 23:
      return V ? launch_dma<T, 64, 64, 2, 2, 2, TA, TB>(g, s)
               : launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 24:
      return V ? launch_dma<T, 64, 32, 2, 2, 3, TA, TB>(g, s)
               : launch_one<T, 64, 32, V, 2, 2, 1, TA, TB>(g, s);
    case 25: return launch_naive<T, TA, TB>(g, s);
    case 26:
      return V ? launch_dma<T, 64, 64, 2, 2, 2, TA, TB, 2>(g, s)
               : launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 27:
      return V ? launch_dma<T, 128, 64, 2, 2, 2, TA, TB, 2>(g, s)
               : launch_one<T, 128, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 28:
      return V ? launch_dma<T, 64, 64, 2, 2, 4, TA, TB, 2>(g, s)
               : launch_one<T, 64, 64, V, 2, 2, 1, TA, TB>(g, s);
    case 29:
      return V ? launch_dma<T, 64, 32, 2, 1, 2, TA, TB, 2>(g, s)
               : launch_one<T, 64, 32, V, 2, 2, 1, TA, TB>(g, s);
  }
  set_error("unknown tile cfg %d", cfg);
  return MG_ERR_INVALID_ARG;
}

template <typename T, bool TA, bool TB>
int gemm_tiles_t(int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                 int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                 hipStream_t s) {
  GemmArgs<T> g;
  g.A = static_cast<const T *>(A);
  g.B = static_cast<const T *>(B);
  g.C = static_cast<T *>(C);
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.m = (int)m;
  g.n = (int)n;
  g.k = (int)k;
  g.alpha = (T)alpha;
  g.beta = (T)beta;
  constexpr int VEC = Mfma<T>::VEC;
  const bool vec_ok = vec_aligned(A, lda, sizeof(T), VEC) &&
                      vec_aligned(B, ldb, sizeof(T), VEC) && vec_aligned(C, ldc, sizeof(T), VEC);
  return vec_ok ? launch_cfg<T, true, TA, TB>(cfg, g, s) : launch_cfg<T, false, TA, TB>(cfg, g, s);
}

}  // namespace

// The tiled kernels for one layout combination (m, n, k >= 1, alpha != 0,
// arguments validated).
template <bool TA, bool TB>
int gemm_tiles(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
               int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
               hipStream_t s) {
  if (dtype == MG_F64)
    return gemm_tiles_t<double, TA, TB>(cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
  return gemm_tiles_t<float, TA, TB>(cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

}  // namespace mg
