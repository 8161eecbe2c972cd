// Native FP64 / FP32 GEMM: one workgroup per macro-tile of C (Section 4.2.2
// tiling), work division chosen per shape on the host.
#include "gemm_native.h"

#include "gemm_dma.h"
#include "gemm_tile.h"

namespace mg {

namespace {

constexpr int kGroupM = 8;  // tile-rows walked together by the raster

template <typename T, int BM, int BN, bool VEC_OK, int WGM, int WGN, int BKM>
__global__ __launch_bounds__((TileShape<T, BM, BN, WGM, WGN, BKM>::THREADS)) void gemm_native_kernel(
    GemmArgs<T> g, int tiles_m, int tiles_n) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *smem = reinterpret_cast<T *>(lds_raw);
  int tm, tn;
  const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  grouped_tile(t, tiles_m, tiles_n, kGroupM, tm, tn);
  gemm_tile<T, BM, BN, VEC_OK, WGM, WGN, BKM>(g, tm * BM, tn * BN, smem);
}

template <typename T, int BM, int BN, int WGM, int WGN, int NS>
__global__ __launch_bounds__((DmaShape<T, BM, BN, WGM, WGN, NS>::THREADS),
                             (DmaShape<T, BM, BN, WGM, WGN, NS>::MINW)) void gemm_dma_kernel(
    GemmArgs<T> g, int tiles_m, int tiles_n) {
  extern __shared__ __align__(16) unsigned char lds[];
  int tm, tn;
  const int t = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  grouped_tile(t, tiles_m, tiles_n, kGroupM, tm, tn);
  gemm_dma_tile<T, BM, BN, WGM, WGN, NS>(g, tm * BM, tn * BN, lds);
}

// C <- beta*C (alpha == 0 or k == 0).  beta == 0 writes zeros without reading.
template <typename T>
__global__ void scale_kernel(T *C, int64_t ldc, int m, int n, T beta) {
  const int64_t total = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    T *p = C + i * ldc + j;
    *p = beta == T(0) ? T(0) : beta * *p;
  }
}

struct CfgDesc {
  int bm, bn, wgm, wgn, bkm;
};
// Work divisions 0-13 stage A and B through registers; 14-24 load them
// straight into an LDS ring (16-byte aligned operands only: otherwise a
// register-staged division of the same macro-tile runs).
// Work divisions: macro-tile, wavefront grid, k-step multiplier.
constexpr CfgDesc kCfgs[] = {{128, 128, 2, 2, 1}, {128, 64, 2, 2, 1}, {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1},   {32, 32, 2, 2, 1},  {128, 128, 4, 2, 1},
                             {128, 128, 2, 4, 1}, {64, 64, 2, 2, 2},  {128, 64, 4, 2, 1},
                             {128, 64, 2, 2, 2},  {256, 128, 4, 2, 1}, {128, 256, 2, 4, 1},
                             {256, 128, 4, 4, 1}, {128, 128, 4, 2, 2},  {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1},   {128, 64, 2, 2, 1},  {128, 128, 2, 4, 1},
                             {256, 128, 4, 4, 1},  {32, 32, 2, 2, 1},   {64, 64, 4, 2, 1},
                             {128, 128, 2, 4, 1},  {128, 128, 2, 2, 1}, {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1}};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

template <typename T, int BM, int BN, bool VEC_OK, int WGM = 2, int WGN = 2, int BKM = 1>
int launch_one(const GemmArgs<T> &g, hipStream_t s) {
  typedef TileShape<T, BM, BN, WGM, WGN, BKM> S;
  const int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  if (tiles > INT32_MAX) {
    set_error("too many tiles (%lld)", (long long)tiles);
    return MG_ERR_INVALID_ARG;
  }
  auto kern = gemm_native_kernel<T, BM, BN, VEC_OK, WGM, WGN, BKM>;
  static bool attr_set = false;  // per template instance
  if (!attr_set) {
    MG_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)S::LDS_BYTES));
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(S::THREADS), S::LDS_BYTES, s, g, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <typename T, int BM, int BN, int WGM, int WGN, int NS>
int launch_dma(const GemmArgs<T> &g, hipStream_t s) {
  typedef DmaShape<T, BM, BN, WGM, WGN, NS> S;
  const int tiles_m = (g.m + BM - 1) / BM, tiles_n = (g.n + BN - 1) / BN;
  const int64_t tiles = (int64_t)tiles_m * tiles_n;
  if (tiles > INT32_MAX) {
    set_error("too many tiles (%lld)", (long long)tiles);
    return MG_ERR_INVALID_ARG;
  }
  auto kern = gemm_dma_kernel<T, BM, BN, WGM, WGN, NS>;
  static bool attr_set = false;  // per template instance
  if (!attr_set) {
    MG_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)S::LDS_BYTES));
    attr_set = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(S::THREADS), S::LDS_BYTES, s, g, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <typename T, bool VEC_OK>
int launch_cfg(int cfg, const GemmArgs<T> &g, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_one<T, 128, 128, VEC_OK>(g, s);
    case 1: return launch_one<T, 128, 64, VEC_OK>(g, s);
    case 2: return launch_one<T, 64, 64, VEC_OK>(g, s);
    case 3: return launch_one<T, 64, 32, VEC_OK>(g, s);
    case 4: return launch_one<T, 32, 32, VEC_OK>(g, s);
    case 5: return launch_one<T, 128, 128, VEC_OK, 4, 2, 1>(g, s);
    case 6: return launch_one<T, 128, 128, VEC_OK, 2, 4, 1>(g, s);
    case 7: return launch_one<T, 64, 64, VEC_OK, 2, 2, 2>(g, s);
    case 8: return launch_one<T, 128, 64, VEC_OK, 4, 2, 1>(g, s);
    case 9: return launch_one<T, 128, 64, VEC_OK, 2, 2, 2>(g, s);
    case 10: return launch_one<T, 256, 128, VEC_OK, 4, 2, 1>(g, s);
    case 11: return launch_one<T, 128, 256, VEC_OK, 2, 4, 1>(g, s);
    case 12: return launch_one<T, 256, 128, VEC_OK, 4, 4, 1>(g, s);
    case 13: return launch_one<T, 128, 128, VEC_OK, 4, 2, 2>(g, s);
    case 14:
      return VEC_OK ? launch_dma<T, 64, 64, 2, 2, 4>(g, s) : launch_one<T, 64, 64, VEC_OK>(g, s);
    case 15:
      return VEC_OK ? launch_dma<T, 64, 32, 2, 2, 4>(g, s) : launch_one<T, 64, 32, VEC_OK>(g, s);
    case 16:
      return VEC_OK ? launch_dma<T, 128, 64, 2, 2, 4>(g, s)
                    : launch_one<T, 128, 64, VEC_OK>(g, s);
    case 17:
      return VEC_OK ? launch_dma<T, 128, 128, 2, 4, 3>(g, s)
                    : launch_one<T, 128, 128, VEC_OK, 4, 2, 2>(g, s);
    case 18:
      return VEC_OK ? launch_dma<T, 256, 128, 4, 4, 3>(g, s)
                    : launch_one<T, 256, 128, VEC_OK, 4, 4, 1>(g, s);
    case 19:
      return VEC_OK ? launch_dma<T, 32, 32, 2, 2, 4>(g, s) : launch_one<T, 32, 32, VEC_OK>(g, s);
    case 20:
      return VEC_OK ? launch_dma<T, 64, 64, 4, 2, 4>(g, s) : launch_one<T, 64, 64, VEC_OK>(g, s);
    case 21:
      return VEC_OK ? launch_dma<T, 128, 128, 2, 4, 2>(g, s)
                    : launch_one<T, 128, 128, VEC_OK, 4, 2, 2>(g, s);
    case 22:
      return VEC_OK ? launch_dma<T, 128, 128, 2, 2, 2>(g, s)
                    : launch_one<T, 128, 128, VEC_OK, 4, 2, 2>(g, s);
    case 23:
      return VEC_OK ? launch_dma<T, 64, 64, 2, 2, 2>(g, s) : launch_one<T, 64, 64, VEC_OK>(g, s);
    case 24:
      return VEC_OK ? launch_dma<T, 64, 32, 2, 2, 3>(g, s) : launch_one<T, 64, 32, VEC_OK>(g, s);
  }
  set_error("unknown tile cfg %d", cfg);
  return MG_ERR_INVALID_ARG;
}

template <typename T>
int gemm_native_t(int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                  int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                  hipStream_t s) {
  if (m == 0 || n == 0) return MG_OK;
  if (alpha == 0.0 || k == 0) {
    const int64_t total = m * n;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_kernel<T>, dim3(blocks), dim3(256), 0, s, static_cast<T *>(C), ldc,
                       (int)m, (int)n, (T)beta);
    MG_HIP_TRY(hipGetLastError());
    return MG_OK;
  }
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
  return vec_ok ? launch_cfg<T, true>(cfg, g, s) : launch_cfg<T, false>(cfg, g, s);
}

}  // namespace

bool vec_aligned(const void *p, int64_t ld, int64_t esz, int vec) {
  return (reinterpret_cast<uintptr_t>(p) % (uintptr_t)(esz * vec)) == 0 && ld % vec == 0;
}

int num_tile_cfgs() { return kNumCfgs; }

int tile_cfg_info(int dtype, int cfg, int *bm, int *bn, int *bk, int *threads) {
  if (cfg < 0 || cfg >= kNumCfgs || (dtype != MG_F64 && dtype != MG_F32)) {
    set_error("unknown tile cfg %d / dtype %d", cfg, dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (bm) *bm = kCfgs[cfg].bm;
  if (bn) *bn = kCfgs[cfg].bn;
  if (bk) *bk = kCfgs[cfg].bkm * (dtype == MG_F64 ? Mfma<double>::BK : Mfma<float>::BK);
  if (threads) *threads = 64 * kCfgs[cfg].wgm * kCfgs[cfg].wgn;
  return MG_OK;
}

int pick_tile_cfg(int dtype, int64_t m, int64_t n, int64_t k) {
  (void)k;
  // Measured on MI355X (16-byte aligned operands): 128x128 tiles with a
  // 2-stage direct-load ring and two workgroups per CU once every CU gets a
  // tile (n >= 2048; FP64 on 8 wavefronts: 90 % of peak at 8192; FP32 on 4
  // wavefronts once there are four tiles per CU), then the 64x64 ring
  // (n = 1024) and the 32x32 ring (n = 512), then the small register-staged
  // tiles.  Unaligned operands run a register-staged division of the same
  // macro-tile.
  auto tiles = [&](int c) { return ceil_div(m, kCfgs[c].bm) * ceil_div(n, kCfgs[c].bn); };
  const int64_t cus = 256;
  if (dtype == MG_F32 && tiles(22) >= 4 * cus) return 22;
  if (tiles(21) >= cus) return 21;
  if (tiles(23) >= cus) return 23;
  if (tiles(19) >= cus) return 19;
  if (tiles(2) >= 2 * cus) return 2;
  if (tiles(3) >= 2 * cus) return 3;
  return 4;
}

int gemm_native(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                hipStream_t s) {
  if (dtype == MG_F64)
    return gemm_native_t<double>(cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
  if (dtype == MG_F32)
    return gemm_native_t<float>(cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
  set_error("unknown dtype %d", dtype);
  return MG_ERR_INVALID_ARG;
}

}  // namespace mg
