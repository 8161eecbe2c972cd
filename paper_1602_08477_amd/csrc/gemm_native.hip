// Native FP64 / FP32 GEMM: one workgroup per macro-tile of C (Section 4.2.2
// tiling), work division chosen per shape on the host.  This unit holds the
// plain-layout kernels and the host side; the transposed layouts are built
// in gemm_op_*.hip.
#include "gemm_launch.h"

namespace mg {

namespace {

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
  int ks = 1;  // k groups of wgm x wgn wavefronts
};
// Work divisions (the order of launch_cfg): macro-tile, wavefront grid,
// k-step multiplier.  0-13 register-staged, 14-24 direct-load rings, 25 the
// naive mapping (a 16 x 16 workgroup of lanes, one output each), 26-29
// direct-load rings with two k groups of wavefronts.
constexpr CfgDesc kCfgs[] = {{128, 128, 2, 2, 1}, {128, 64, 2, 2, 1}, {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1},   {32, 32, 2, 2, 1},  {128, 128, 4, 2, 1},
                             {128, 128, 2, 4, 1}, {64, 64, 2, 2, 2},  {128, 64, 4, 2, 1},
                             {128, 64, 2, 2, 2},  {256, 128, 4, 2, 1}, {128, 256, 2, 4, 1},
                             {256, 128, 4, 4, 1}, {128, 128, 4, 2, 2},  {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1},   {128, 64, 2, 2, 1},  {128, 128, 2, 4, 1},
                             {256, 128, 4, 4, 1},  {32, 32, 2, 2, 1},   {64, 64, 4, 2, 1},
                             {128, 128, 2, 4, 1},  {128, 128, 2, 2, 1}, {64, 64, 2, 2, 1},
                             {64, 32, 2, 2, 1},   {16, 16, 0, 0, 0},  {64, 64, 2, 2, 1, 2},
                             {128, 64, 2, 2, 1, 2}, {64, 64, 2, 2, 1, 2},  {64, 32, 2, 1, 1, 2}};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kNaiveCfg = 25;  // one output per lane, no LDS (wgm/wgn/bkm unused)

template <typename T>
int scale_c(int64_t m, int64_t n, double beta, void *C, int64_t ldc, hipStream_t s) {
  const int64_t total = m * n;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(scale_kernel<T>, dim3(blocks), dim3(256), 0, s, static_cast<T *>(C), ldc,
                     (int)m, (int)n, (T)beta);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
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
  if (cfg == kNaiveCfg) {
    if (bk) *bk = 1;
    if (threads) *threads = kCfgs[cfg].bm * kCfgs[cfg].bn;
    return MG_OK;
  }
  if (bk) *bk = kCfgs[cfg].bkm * (dtype == MG_F64 ? Mfma<double>::BK : Mfma<float>::BK);
  if (threads) *threads = 64 * kCfgs[cfg].wgm * kCfgs[cfg].wgn * kCfgs[cfg].ks;
  return MG_OK;
}

int pick_tile_cfg(int dtype, int64_t m, int64_t n, int64_t k) {
  (void)k;
  // Measured on MI355X (16-byte aligned operands), FP64: the 128x128 ring on
  // 8 wavefronts once it gives every CU two tiles (90 % of peak at 8192);
  // below that the 64x64 ring on 4 wavefronts while it still gives every CU
  // three or more tiles (n = 2048: 64.7 TFLOP/s against 64.1 for 128x128;
  // n = 2560: 58.7 against 54.2); then the 64x32 ring with two k groups of
  // wavefronts while it gives every CU four tiles (n = 1536: 49.9 against
  // 44.6), the 64x64 one with two k groups (n = 1024: 44-47 against 41-43);
  // then the 32x32 ring (n = 512).
  // FP32: the 128x128 ring on 4 wavefronts from four tiles per CU, on 8
  // from one, then the same smaller tiles.  Below those the small
  // register-staged tiles; unaligned operands run a register-staged
  // division of the same macro-tile.
  auto tiles = [&](int c) { return ceil_div(m, kCfgs[c].bm) * ceil_div(n, kCfgs[c].bn); };
  const int64_t cus = 256;
  if (dtype == MG_F32) {
    if (tiles(22) >= 4 * cus) return 22;
    if (tiles(21) >= cus) return 21;
  } else {
    if (tiles(21) >= 2 * cus) return 21;
    if (tiles(23) >= 3 * cus) return 23;
    if (tiles(29) >= 4 * cus) return 29;
  }
  if (tiles(26) >= cus) return 26;
  if (tiles(19) >= cus) return 19;
  if (tiles(2) >= 2 * cus) return 2;
  if (tiles(3) >= 2 * cus) return 3;
  return 4;
}

int gemm_tiles_nn(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha,
                  const void *A, int64_t lda, const void *B, int64_t ldb, double beta, void *C,
                  int64_t ldc, hipStream_t s) {
  return gemm_tiles<false, false>(dtype, cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

int gemm_native_op(int dtype, int cfg, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                   double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                   double beta, void *C, int64_t ldc, hipStream_t s) {
  if (dtype != MG_F64 && dtype != MG_F32) {
    set_error("unknown dtype %d", dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (m == 0 || n == 0) return MG_OK;
  if (alpha == 0.0 || k == 0)
    return dtype == MG_F64 ? scale_c<double>(m, n, beta, C, ldc, s)
                           : scale_c<float>(m, n, beta, C, ldc, s);
  auto run = ta ? (tb ? gemm_tiles_tt : gemm_tiles_tn) : (tb ? gemm_tiles_nt : gemm_tiles_nn);
  return run(dtype, cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

int gemm_native(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                hipStream_t s) {
  return gemm_native_op(dtype, cfg, false, false, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

}  // namespace mg
