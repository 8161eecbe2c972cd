// Split-precision FP64 GEMM on INT8 / BF16 matrix cores.
//
// The method (an error-free splitting in the style of Ozaki et al.; not part
// of the Alpaka paper, which computes DGEMM natively):
//  1. E_i = frexp exponent of max_p |A[i,p]| (so |A[i,:]| < 2^E_i), F_j the
//     same for column j of B; zero rows/columns get 0.
//  2. r = x * 2^-E;  for t = 1..s:  y = r * 2^b,  slice_t = trunc(y),
//     r = y - slice_t.  All exact; |slice| <= 2^b - 1 (b = 7 for INT8,
//     b = 8 for BF16, whose 8-bit significand holds such integers exactly).
//  3. P_d = sum_{p+q=d} A_p B_q for d = 2..s+1 (exact integers: INT32
//     accumulation for INT8; FP32 accumulation over 256-long k chunks, then
//     INT32, for BF16).
//  4. acc = sum_d P_d 2^(-b d) in FP64 (increasing d);
//     C = alpha * 2^(E_i+F_j) acc + beta * C.
// The workspace holds E, F and the slices, padded to 128 in every extent
// with zeros so that the product kernel runs without bounds checks.
#include "split.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <numeric>
#include <utility>
#include <vector>

#include "gemm_native.h"

namespace mg {

namespace {

constexpr int kStageBytes = 128;  // k bytes of one slice row per LDS stage
constexpr int kPitch = kStageBytes + 16;  // LDS row pitch: conflict-free b128 reads

__device__ __forceinline__ int exp_of(double x) {
  if (x == 0.0) return INT_MIN;
  int e;
  (void)frexp(x, &e);
  return e;
}

// ------------------------------------------------------------ step 1: scales
// The preparation kernels are written as bodies over a block index so that
// the single-problem launches and the batched launches (one grid over the
// blocks of many problems) run the same code.  All use 256 threads.
__device__ __forceinline__ void fill_int_body(int *p, int count, int v, int block) {
  const int i = block * 256 + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void fill_int_kernel(int *p, int count, int v) {
  fill_int_body(p, count, v, blockIdx.x);
}

constexpr int kColRows = 64;  // rows of B per thread in col_exp_body

// Column exponents of B for the 256 columns of block `bx`, over the k chunks
// by, by + gy, ... (the maximum is order-independent).
__device__ __forceinline__ void col_exp_body(const double *B, int64_t ldb, int k, int n, int *F,
                                             int bx, int by, int gy) {
  const int j = bx * 256 + threadIdx.x;
  if (j >= n) return;
  const int nchunks = (k + kColRows - 1) / kColRows;
  for (int ch = by; ch < nchunks; ch += gy) {
    int e = INT_MIN;
    const int r1 = min(k, (ch + 1) * kColRows);
#pragma unroll 8
    for (int r = ch * kColRows; r < r1; ++r) e = max(e, exp_of(B[(int64_t)r * ldb + j]));
    if (e != INT_MIN) atomicMax(F + j, e);
  }
}


// ------------------------------------------------------------ step 2: slices
// Packs CW slice values (CW*ESZ == 16 bytes) into one 16-byte store.
template <int ESZ>
struct SlicePack;

template <>
struct SlicePack<1> {  // INT8
  static constexpr int CW = 16;
  __device__ static __forceinline__ i4v pack(const int *q) {
    i4v o;
#pragma unroll
    for (int w = 0; w < 4; ++w)
      o[w] = (q[4 * w] & 0xff) | ((q[4 * w + 1] & 0xff) << 8) | ((q[4 * w + 2] & 0xff) << 16) |
             ((q[4 * w + 3] & 0xff) << 24);
    return o;
  }
};

template <>
struct SlicePack<2> {  // BF16: an integer |q| <= 256 is exact in bf16 = top half of its float
  static constexpr int CW = 8;
  __device__ static __forceinline__ unsigned bf16_bits(int q) {
    return __float_as_uint((float)q) >> 16;
  }
  __device__ static __forceinline__ i4v pack(const int *q) {
    i4v o;
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = (int)(bf16_bits(q[2 * w]) | (bf16_bits(q[2 * w + 1]) << 16));
    return o;
  }
};

// One slicing round on CW values: y = r*2^b, q = trunc(y), r = y - q.
template <int CW>
__device__ __forceinline__ void slice_round(double *r, int *q, int bits) {
#pragma unroll
  for (int e = 0; e < CW; ++e) {
    const double y = ldexp(r[e], bits);
    const double t = trunc(y);
    q[e] = (int)t;
    r[e] = y - t;
  }
}

// Steps 1 and 2 for A in one pass: one workgroup per (padded) row finds the
// row's exponent and slices it, so A is read from HBM once.  A thread owns
// quads (4 consecutive k) tid, tid+256, ...; rows up to 4096 long stay in
// registers between the two passes, longer rows are read again (from L2).
template <int ESZ>
__device__ __forceinline__ void slice_rows_exp_body(const double *A, int64_t lda, int m, int k,
                                                    int mp, int64_t kp, int *E, int s, int bits,
                                                    unsigned char *out, int i) {
  constexpr int QPT = 4;  // quads per thread held in registers
  const int tid = threadIdx.x;
  const bool live = i < m;
  const double *row = A + (int64_t)(live ? i : 0) * lda;
  const int64_t quads = kp / 4;
  const bool regs = quads <= 256 * QPT;
  auto load = [&](int64_t kk) { return (live && kk < k) ? row[kk] : 0.0; };
  double x[QPT][4];
  int e = INT_MIN;
  for (int64_t q0 = 0; q0 < quads; q0 += 256 * QPT) {
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      const int64_t qd = q0 + tid + 256 * j;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double val = qd < quads ? load(qd * 4 + v) : 0.0;
        x[j][v] = val;
        e = max(e, exp_of(val));
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e = max(e, __shfl_xor(e, off));
  __shared__ int red[4];
  if ((tid & 63) == 0) red[tid >> 6] = e;
  __syncthreads();
  e = max(max(red[0], red[1]), max(red[2], red[3]));
  const int ei = (e == INT_MIN) ? 0 : e;
  if (tid == 0) E[i] = ei;
  const int64_t slice_bytes = (int64_t)mp * kp * ESZ;
  for (int64_t q0 = 0; q0 < quads; q0 += 256 * QPT) {
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
      const int64_t qd = q0 + tid + 256 * j;
      if (qd >= quads) continue;
      double r[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) r[v] = ldexp(regs ? x[j][v] : load(qd * 4 + v), -ei);
      unsigned char *o = out + ((int64_t)i * kp + qd * 4) * ESZ;
      for (int t = 0; t < s; ++t) {
        int q[4];
        slice_round<4>(r, q, bits);
        if (ESZ == 1) {
          const unsigned w = (q[0] & 0xff) | ((q[1] & 0xff) << 8) | ((q[2] & 0xff) << 16) |
                             ((unsigned)(q[3] & 0xff) << 24);
          *reinterpret_cast<unsigned *>(o + t * slice_bytes) = w;
        } else {
          uint2 w;
          w.x = SlicePack<2>::bf16_bits(q[0]) | (SlicePack<2>::bf16_bits(q[1]) << 16);
          w.y = SlicePack<2>::bf16_bits(q[2]) | (SlicePack<2>::bf16_bits(q[3]) << 16);
          *reinterpret_cast<uint2 *>(o + t * slice_bytes) = w;
        }
      }
    }
  }
}

// The same for rows of at most 16 * LPR (padded) k with LPR lanes per row
// (LPR = 16, 32 or 64: 4, 2 or 1 rows per wavefront): a lane holds quads l,
// l + LPR, l + 2 LPR, l + 3 LPR of its row in registers (l = its index in
// the row's lane group), and the row's exponent is a reduction over the
// group.  This lane's row is `i`.
template <int ESZ, int LPR>
__device__ __forceinline__ void slice_rows_wave_body(const double *A, int64_t lda, int m, int k,
                                                     int mp, int64_t kp, int *E, int s, int bits,
                                                     unsigned char *out, int i) {
  static_assert(LPR == 16 || LPR == 32 || LPR == 64, "lanes per row");
  constexpr int QPT = 4;
  const int lane = threadIdx.x & (LPR - 1);
  const bool live = i < m;
  const double *row = A + (int64_t)(live ? i : 0) * lda;
  const int quads = (int)(kp / 4);
  double x[QPT][4];
  int e = INT_MIN;
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int qd = lane + LPR * j;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int kk = qd * 4 + v;
      const double val = (live && qd < quads && kk < k) ? row[kk] : 0.0;
      x[j][v] = val;
      e = max(e, exp_of(val));
    }
  }
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) e = max(e, __shfl_xor(e, off));
  const int ei = (e == INT_MIN) ? 0 : e;
  if (lane == 0) E[i] = ei;
  const int64_t slice_bytes = (int64_t)mp * kp * ESZ;
#pragma unroll
  for (int j = 0; j < QPT; ++j) {
    const int qd = lane + LPR * j;
    if (qd >= quads) continue;
    double r[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = ldexp(x[j][v], -ei);
    unsigned char *o = out + ((int64_t)i * kp + qd * 4) * ESZ;
    for (int t = 0; t < s; ++t) {
      int q[4];
      slice_round<4>(r, q, bits);
      if (ESZ == 1) {
        const unsigned w = (q[0] & 0xff) | ((q[1] & 0xff) << 8) | ((q[2] & 0xff) << 16) |
                           ((unsigned)(q[3] & 0xff) << 24);
        *reinterpret_cast<unsigned *>(o + t * slice_bytes) = w;
      } else {
        uint2 w;
        w.x = SlicePack<2>::bf16_bits(q[0]) | (SlicePack<2>::bf16_bits(q[1]) << 16);
        w.y = SlicePack<2>::bf16_bits(q[2]) | (SlicePack<2>::bf16_bits(q[3]) << 16);
        *reinterpret_cast<uint2 *>(o + t * slice_bytes) = w;
      }
    }
  }
}

// Steps 1 and 2 without B's slices in one launch: blocks [0, cx*cy) find
// B's column exponents (col_exp_body), the rest each find one row's
// exponent of A and slice it.  The two passes are independent, so they run
// side by side instead of one after the other.
template <int ESZ>
__global__ __launch_bounds__(256) void exp_rows_kernel(const double *A, int64_t lda, int m, int k,
                                                       int mp, int64_t kp, int *E, int s, int bits,
                                                       unsigned char *out, const double *B,
                                                       int64_t ldb, int n, int *F, int cx,
                                                       int cy) {
  const int b = (int)blockIdx.x, ncol = cx * cy;
  if (b < ncol) col_exp_body(B, ldb, k, n, F, b % cx, b / cx, cy);
  else slice_rows_exp_body<ESZ>(A, lda, m, k, mp, kp, E, s, bits, out, b - ncol);
}

// B slices, stored transposed [s][np][kp] (k contiguous per column of B):
// a 64 x 64 block of B is transposed through LDS.
template <int ESZ>
__device__ __forceinline__ void slice_cols_body(const double *B, int64_t ldb, int k, int n,
                                                int np, int64_t kp, int *F, int s, int bits,
                                                unsigned char *out, int block) {
  // (Measured alternatives: one wavefront per 16-long k range reading 64
  // consecutive columns has no LDS bank conflicts but writes 16-byte pieces
  // of 64 columns, 25 % slower in the 2000-problem batch; rotating T's
  // columns per 16-row block left the conflict count unchanged.)
  __shared__ double T[64][65];
  const int64_t kblocks = kp / 64;
  const int j0 = (int)(block / kblocks) * 64;
  const int64_t k0 = (block % kblocks) * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int kk = e >> 6, jj = e & 63;
    const int64_t gk = k0 + kk;
    const int gj = j0 + jj;
    T[kk][jj] = (gk < k && gj < n) ? B[gk * ldb + gj] : 0.0;
  }
  __syncthreads();
  // column jj, 16-long k range kq: the 4 lanes of a column write its 64
  // contiguous bytes of each slice
  const int jj = tid >> 2, kq = tid & 3;
  const int j = j0 + jj;
  // F[j] still holds INT_MIN for an all-zero (or padding) column: its scale
  // is 0, and the first k-block of the column stores that back for the
  // product kernel's epilogue.
  const int fraw = F[j];
  const int fj = fraw == INT_MIN ? 0 : fraw;
  if (k0 == 0 && kq == 0 && fraw == INT_MIN) F[j] = 0;
  double r[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) r[e] = ldexp(T[kq * 16 + e][jj], -fj);
  constexpr int CW = SlicePack<ESZ>::CW;
  const int64_t slice_bytes = (int64_t)np * kp * ESZ;
  unsigned char *o = out + ((int64_t)j * kp + k0 + kq * 16) * ESZ;
  for (int t = 0; t < s; ++t) {
    int q[16];
    slice_round<16>(r, q, bits);
#pragma unroll
    for (int h = 0; h < 16 / CW; ++h)
      *reinterpret_cast<i4v *>(o + t * slice_bytes + h * 16) = SlicePack<ESZ>::pack(q + h * CW);
  }
}

template <int ESZ>
__global__ __launch_bounds__(256) void slice_cols_kernel(const double *B, int64_t ldb, int k, int n,
                                                         int np, int64_t kp, int *F, int s,
                                                         int bits, unsigned char *out) {
  slice_cols_body<ESZ>(B, ldb, k, n, np, kp, F, s, bits, out, blockIdx.x);
}

// ------------------------------------------------- steps 3-4: slice products
template <int ALGO>
struct SplitMma;

template <>
struct SplitMma<MG_SPLIT_I8> {
  typedef i4v acc_t;
  static constexpr int CHUNK_STAGES = 0;  // INT32 accumulates a diagonal directly
  __device__ static __forceinline__ acc_t mma(i4v a, i4v b, acc_t c) {
    return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
  }
};

template <>
struct SplitMma<MG_SPLIT_BF16> {
  typedef f4v acc_t;
  static constexpr int CHUNK_STAGES = 4;  // 256 k: 256 * 255^2 < 2^24 keeps FP32 exact
  __device__ static __forceinline__ acc_t mma(i4v a, i4v b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a),
                                                   __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
  }
};

struct SplitArgs {
  const unsigned char *As, *Bs;
  const int *E, *F;
  double *P;  // FP64 partial sums [mp][np]
  int32_t *Q; // pair-parallel division: INT32 partial diagonal sums (in P's region)
  double *C;
  int64_t ldc;
  int m, n, mp, np;
  int64_t kp_bytes;  // row pitch of a slice in bytes
  int s, bits;
  int seg_stages, total_stages;
  double alpha, beta;
};

struct Step {
  int seg, d, p, st;
};

__device__ __forceinline__ int pmax_of(int d, int s) { return min(s, d - 1); }

__device__ __forceinline__ int seg_len(int seg, const SplitArgs &a) {
  return min(a.seg_stages, a.total_stages - seg * a.seg_stages);
}

// Next (segment, diagonal, pair, stage) in the order the kernel walks them.
__device__ __forceinline__ void advance(Step &x, const SplitArgs &a) {
  if (++x.st < seg_len(x.seg, a)) return;
  x.st = 0;
  if (++x.p <= pmax_of(x.d, a.s)) return;
  if (++x.d > a.s + 1) {
    x.d = 2;
    ++x.seg;
  }
  x.p = max(1, x.d - a.s);
}

// Partial sums of step 4 live in the workspace tile-major and lane-contiguous:
// element e of lane t of tile b at P[b*BM*BN + e*THREADS + t], so each
// fold reads and writes whole contiguous rows of lanes with constant offsets.
// Element e = (i*FNW + j)*4 + r is output row 16i + 4g + r, column 16j + l16
// of the wave's sub-tile (g = lane/16, l16 = lane%16).
// Blocks of a row folded / stored per memory round trip (4 FP64 values each):
// two at most, one for tiles of 16 blocks per wave, so that the gathered
// values fit the register budget of the largest tiles.
template <int FMW, int FNW>
constexpr int kFoldChunk = FMW * FNW >= 16 ? 1 : (FNW > 2 ? 2 : FNW);

template <typename M, int FMW, int FNW, int THREADS>
__device__ __forceinline__ void fold_partials(typename M::acc_t (&acc)[FMW][FNW],
                                              i4v (&dacc)[FMW][FNW], double *plane, double sc,
                                              bool first) {
  // Opaque copy of the base: keeps the compiler from hoisting all FMW*FNW*4
  // element addresses out of the k loop (64-bit each, they would not fit).
  asm volatile("" : "+v"(plane));
  constexpr int CJ = kFoldChunk<FMW, FNW>;
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j0 = 0; j0 < FNW; j0 += CJ) {
      // the chunk's loads first (one memory round trip), then the fused
      // multiply-adds and stores
      double part[CJ][4];
#pragma unroll
      for (int j = 0; j < CJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[j][r] = first ? 0.0 : plane[((i * FNW + j0 + j) * 4 + r) * THREADS];
#pragma unroll
      for (int j = 0; j < CJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int v = M::CHUNK_STAGES > 0 ? dacc[i][j0 + j][r] : (int)acc[i][j0 + j][r];
          plane[((i * FNW + j0 + j) * 4 + r) * THREADS] = fma((double)v, sc, part[j][r]);
          dacc[i][j0 + j][r] = 0;
          if (M::CHUNK_STAGES == 0) acc[i][j0 + j][r] = 0;
        }
      // one chunk in flight at a time: bounds the live FP64 registers
      __builtin_amdgcn_sched_barrier(0);
    }
}

// C = alpha * 2^(E_i + F_j) * fin + beta * C for one block of this lane's
// outputs (rows rowb .. rowb+3, columns col0 + 16j), each product and the sum
// rounded once.  Every operand (E, F, and C when beta != 0) is loaded first,
// from addresses clamped into the matrix, so the loads are in flight
// together (one memory round trip, not one per output); values of rows or
// columns outside the matrix are computed and not stored.
template <int FNW>
__device__ __forceinline__ void store_block(const SplitArgs &a, const double (&fin)[4][FNW],
                                            int rowb, int col0) {
  int er[4], fc[FNW], cc[FNW];
  int64_t roff[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = min(rowb + r, a.m - 1);
    er[r] = a.E[row];
    roff[r] = (int64_t)row * a.ldc;
  }
#pragma unroll
  for (int j = 0; j < FNW; ++j) {
    cc[j] = min(col0 + 16 * j, a.n - 1);
    fc[j] = a.F[cc[j]];
  }
  const bool with_c = a.beta != 0.0;
  double cv[4][FNW];
  if (with_c) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < FNW; ++j) cv[r][j] = a.C[roff[r] + cc[j]];
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int j = 0; j < FNW; ++j) {
      const double prod = ldexp(fin[r][j], er[r] + fc[j]);
      double o = __dmul_rn(a.alpha, prod);
      if (with_c) o = __dadd_rn(o, __dmul_rn(a.beta, cv[r][j]));
      if (rowb + r < a.m && col0 + 16 * j < a.n) a.C[roff[r] + cc[j]] = o;
    }
}

// Last fold, then the epilogue.  (row0, col0): this lane's first output.
template <typename M, int FMW, int FNW, int THREADS>
__device__ __forceinline__ void finish_tile(const SplitArgs &a, typename M::acc_t (&acc)[FMW][FNW],
                                            i4v (&dacc)[FMW][FNW], const double *plane,
                                            bool only, int row0, int col0) {
  const double sc = ldexp(1.0, -a.bits * (a.s + 1));
  asm volatile("" : "+v"(plane));
  constexpr int CJ = kFoldChunk<FMW, FNW>;
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j0 = 0; j0 < FNW; j0 += CJ) {
      double fin[4][CJ];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
          const int v = M::CHUNK_STAGES > 0 ? dacc[i][j0 + j][r] : (int)acc[i][j0 + j][r];
          const double part = only ? 0.0 : plane[((i * FNW + j0 + j) * 4 + r) * THREADS];
          fin[r][j] = fma((double)v, sc, part);
        }
      store_block<CJ>(a, fin, row0 + 16 * i, col0 + 16 * j0);
      __builtin_amdgcn_sched_barrier(0);
    }
}

// Work divisions of the product kernel: WGM x WGN wavefronts, each owning
// FMW x FNW blocks of 16x16 outputs.
template <int WGM, int WGN, int FMW, int FNW>
struct SplitShape {
  static constexpr int THREADS = 64 * WGM * WGN;
  static constexpr int BM = WGM * 16 * FMW, BN = WGN * 16 * FNW;
  static constexpr int STAGE = (BM + BN) * kPitch;  // bytes of one LDS stage
  static constexpr size_t LDS_BYTES = 2 * (size_t)STAGE;
  static constexpr int NA = BM * (kStageBytes / 16) / THREADS;  // 16-byte chunks per thread
  static constexpr int NB = BN * (kStageBytes / 16) / THREADS;
  static_assert(NA * THREADS == BM * (kStageBytes / 16) && NB * THREADS == BN * (kStageBytes / 16),
                "whole chunks per thread");
};

template <int ALGO, int WGM, int WGN, int FMW, int FNW, int MINB>
__global__ __launch_bounds__((SplitShape<WGM, WGN, FMW, FNW>::THREADS), MINB) void split_gemm_kernel(
    SplitArgs a, int tiles_m, int tiles_n) {
  typedef SplitMma<ALGO> M;
  typedef typename M::acc_t Acc;
  typedef SplitShape<WGM, WGN, FMW, FNW> S;
  constexpr int BM = S::BM, BN = S::BN, STAGE = S::STAGE;
  constexpr int CPR = kStageBytes / 16;  // 16-byte chunks per slice row and stage
  extern __shared__ __align__(16) unsigned char lds[];

  int tm, tn;
  grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * 16 * FMW, wn0 = (wave % WGN) * 16 * FNW;
  const int g = lane >> 4, l16 = lane & 15;

  const int64_t a_slice = (int64_t)a.mp * a.kp_bytes, b_slice = (int64_t)a.np * a.kp_bytes;
  // 16-byte chunk q = tid + THREADS*u of a stage: row q / CPR, byte (q % CPR) * 16.
  int arow[S::NA], acol[S::NA], brow[S::NB], bcol[S::NB];
#pragma unroll
  for (int u = 0; u < S::NA; ++u) {
    const int q = tid + S::THREADS * u;
    arow[u] = q / CPR;
    acol[u] = (q % CPR) * 16;
  }
#pragma unroll
  for (int u = 0; u < S::NB; ++u) {
    const int q = tid + S::THREADS * u;
    brow[u] = q / CPR;
    bcol[u] = (q % CPR) * 16;
  }
  const unsigned char *abase = a.As + (int64_t)m0 * a.kp_bytes;
  const unsigned char *bbase = a.Bs + (int64_t)n0 * a.kp_bytes;
  double *plane = a.P + (int64_t)blockIdx.x * (BM * BN) + tid;  // this lane's partial sums

  i4v ra[S::NA], rb[S::NB];
  auto load = [&](const Step &x) {
    const int64_t koff = (int64_t)(x.seg * a.seg_stages + x.st) * kStageBytes;
    const unsigned char *pa = abase + (x.p - 1) * a_slice + koff;
    const unsigned char *pb = bbase + (x.d - x.p - 1) * b_slice + koff;
#pragma unroll
    for (int u = 0; u < S::NA; ++u)
      ra[u] = *reinterpret_cast<const i4v *>(pa + arow[u] * a.kp_bytes + acol[u]);
#pragma unroll
    for (int u = 0; u < S::NB; ++u)
      rb[u] = *reinterpret_cast<const i4v *>(pb + brow[u] * a.kp_bytes + bcol[u]);
  };
  auto store = [&](int stage) {
    unsigned char *As = lds + stage * STAGE;
    unsigned char *Bs = As + BM * kPitch;
#pragma unroll
    for (int u = 0; u < S::NA; ++u)
      *reinterpret_cast<i4v *>(As + arow[u] * kPitch + acol[u]) = ra[u];
#pragma unroll
    for (int u = 0; u < S::NB; ++u)
      *reinterpret_cast<i4v *>(Bs + brow[u] * kPitch + bcol[u]) = rb[u];
  };

  Acc acc[FMW][FNW];
  i4v dacc[FMW][FNW];  // BF16 only: exact INT32 diagonal sum of FP32 chunk results
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j = 0; j < FNW; ++j) {
      acc[i][j] = Acc{};
      dacc[i][j] = i4v{};
    }

  const int pairs = a.s * (a.s + 1) / 2;
  const int T = pairs * a.total_stages;
  Step cur = {0, 2, 1, 0};
  MG_LDS_POISON_STAGE(lds, 2 * STAGE);
  load(cur);
  store(0);
  __syncthreads();
  for (int t = 0; t < T; ++t) {
    // the other buffer is refilled after this step's products
    MG_LDS_POISON_STAGE(lds + ((t + 1) & 1) * STAGE, STAGE);
    Step nxt = cur;
    advance(nxt, a);
    if (t + 1 < T) load(nxt);
    const unsigned char *As = lds + (t & 1) * STAGE;
    const unsigned char *Bs = As + BM * kPitch;
#pragma unroll
    for (int h = 0; h < kStageBytes / 64; ++h) {
      i4v fa[FMW], fb[FNW];
#pragma unroll
      for (int i = 0; i < FMW; ++i)
        fa[i] = *reinterpret_cast<const i4v *>(As + (wm0 + 16 * i + l16) * kPitch + h * 64 + g * 16);
#pragma unroll
      for (int j = 0; j < FNW; ++j)
        fb[j] = *reinterpret_cast<const i4v *>(Bs + (wn0 + 16 * j + l16) * kPitch + h * 64 + g * 16);
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j) acc[i][j] = M::mma(fa[i], fb[j], acc[i][j]);
    }
    const bool seg_last = cur.st + 1 == seg_len(cur.seg, a);
    if (M::CHUNK_STAGES > 0 && ((cur.st + 1) % (M::CHUNK_STAGES > 0 ? M::CHUNK_STAGES : 1) == 0 ||
                                seg_last)) {
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dacc[i][j][r] += (int)acc[i][j][r];
            acc[i][j][r] = 0;
          }
    }
    // End of a diagonal (within a k segment), except the very last step:
    // fold P_d * 2^(-b d) into this lane's FP64 partial sums.  Each lane only
    // ever touches its own partial-sum addresses, so program order suffices.
    if (t + 1 < T && seg_last && cur.p == pmax_of(cur.d, a.s))
      fold_partials<M, FMW, FNW, S::THREADS>(acc, dacc, plane, ldexp(1.0, -a.bits * cur.d),
                                             cur.seg == 0 && cur.d == 2);
    if (t + 1 < T) store((t + 1) & 1);
    __syncthreads();
    cur = nxt;
  }

  // Last diagonal of the last segment, then the epilogue.
  const bool only = a.s == 1 && a.seg_stages >= a.total_stages;  // a single fold in all
  finish_tile<M, FMW, FNW, S::THREADS>(a, acc, dacc, plane, only, m0 + wm0 + 4 * g,
                                       n0 + wn0 + l16);
}

// ---------------------------------------------------------------------------
// Variant with direct global->LDS loads (gfx950 global_load_lds_dwordx4) into
// an NS-stage ring, so NS-1 stages of slice data are in flight while the
// matrix cores work on the current one, without staging registers.
// LDS rows are SB (64 or 128) bytes without padding.  The 16-byte chunk c of
// row r is stored at chunk c ^ swz(r), swz(r) = (r >> 1) & 7 for 128-byte rows
// and (r >> 1) & 3 for 64-byte rows, so that the rows of a fragment read (16
// consecutive rows, one logical chunk each) fall on different banks; the DMA
// writes are 1 KB contiguous per wave instruction.  Measured with the LDS
// bank-conflict counter: 0 for both row sizes (with (r >> 2) & 3 for 64-byte
// rows, about 4 conflict cycles per fragment read).
template <int WGM, int WGN, int FMW, int FNW, int NS, int SB>
struct SplitDmaShape {
  static constexpr int THREADS = 64 * WGM * WGN;
  static constexpr int WAVES = WGM * WGN;
  static constexpr int BM = WGM * 16 * FMW, BN = WGN * 16 * FNW;
  static constexpr int STAGE = (BM + BN) * SB;  // bytes
  static constexpr size_t LDS_BYTES = (size_t)NS * STAGE;
  static constexpr int CPR = SB / 16;         // chunks per row
  static constexpr int RPI = 64 / CPR;        // rows per DMA instruction (1 KB)
  static constexpr int IA = BM / RPI / WAVES;  // DMA instructions per wave, A
  static constexpr int IB = BN / RPI / WAVES;
  // Two workgroups per CU when their rings fit: the register budget must
  // then allow 2*WAVES/4 wavefronts per SIMD (second __launch_bounds__ value).
  static constexpr int MINW = 2 * LDS_BYTES <= 160 * 1024 ? (WAVES >= 2 ? WAVES / 2 : 1) : 1;
  static_assert(SB == 64 || SB == 128, "stage depth");
  static_assert(IA * RPI * WAVES == BM && IB * RPI * WAVES == BN, "whole DMA rows per wave");
  static_assert(NS >= 2, "at least double buffering");
};

template <int SB>
__device__ __forceinline__ int swz_chunk(int row, int chunk) {
  return SB == 128 ? chunk ^ ((row >> 1) & 7) : chunk ^ ((row >> 1) & 3);
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 s_waitcnt encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[15:14]
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// One 16-byte-per-lane direct load: lane l's chunk lands at lds_row_block + 16*l.
__device__ __forceinline__ void dma16(const unsigned char *src, unsigned char *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0,
                                   0);
}

// One output tile (m0, n0) of the product: every slice pair over every k
// stage, the folds, the epilogue.  `plane0`: the tile's BM*BN partial sums.
// `a.seg_stages` and `a.total_stages` count SB-byte stages here.
template <int ALGO, int WGM, int WGN, int FMW, int FNW, int NS, int SB>
__device__ __forceinline__ void split_dma_tile(const SplitArgs &a, int m0, int n0, double *plane0,
                                               unsigned char *lds) {
  typedef SplitMma<ALGO> M;
  typedef typename M::acc_t Acc;
  typedef SplitDmaShape<WGM, WGN, FMW, FNW, NS, SB> S;
  // FP32 chunk of 256 k for BF16 (512 bytes), in stages
  constexpr int CHUNK = M::CHUNK_STAGES > 0 ? 512 / SB : 0;
  constexpr int BM = S::BM, STAGE = S::STAGE;
  constexpr int DPS = S::IA + S::IB;  // DMA instructions per step per wave
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * 16 * FMW, wn0 = (wave % WGN) * 16 * FNW;
  const int g = lane >> 4, l16 = lane & 15;

  const int64_t a_slice = (int64_t)a.mp * a.kp_bytes, b_slice = (int64_t)a.np * a.kp_bytes;
  // DMA source offsets of this lane: instruction u covers RPI rows starting at
  // RPI*(wave*I + u); the lane supplies row +lane/CPR, physical chunk lane%CPR,
  // which holds logical chunk swz_chunk(row, lane%CPR).
  int64_t asrc[S::IA], bsrc[S::IB];
#pragma unroll
  for (int u = 0; u < S::IA; ++u) {
    const int row = S::RPI * (wave * S::IA + u) + lane / S::CPR;
    asrc[u] = (int64_t)(m0 + row) * a.kp_bytes + swz_chunk<SB>(row, lane % S::CPR) * 16;
  }
#pragma unroll
  for (int u = 0; u < S::IB; ++u) {
    const int row = S::RPI * (wave * S::IB + u) + lane / S::CPR;
    bsrc[u] = (int64_t)(n0 + row) * a.kp_bytes + swz_chunk<SB>(row, lane % S::CPR) * 16;
  }
  double *plane = plane0 + tid;  // this lane's partial sums

  auto issue = [&](const Step &x, int stage) {
    const int64_t koff = (int64_t)(x.seg * a.seg_stages + x.st) * SB;
    const unsigned char *pa = a.As + (x.p - 1) * a_slice + koff;
    const unsigned char *pb = a.Bs + (x.d - x.p - 1) * b_slice + koff;
    unsigned char *la = lds + stage * STAGE;
    unsigned char *lb = la + BM * SB;
#pragma unroll
    for (int u = 0; u < S::IA; ++u) dma16(pa + asrc[u], la + (wave * S::IA + u) * 1024);
#pragma unroll
    for (int u = 0; u < S::IB; ++u) dma16(pb + bsrc[u], lb + (wave * S::IB + u) * 1024);
  };

  Acc acc[FMW][FNW];
  i4v dacc[FMW][FNW];
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j = 0; j < FNW; ++j) {
      acc[i][j] = Acc{};
      dacc[i][j] = i4v{};
    }

  const int pairs = a.s * (a.s + 1) / 2;
  const int T = pairs * a.total_stages;
  Step cur = {0, 2, 1, 0};
  Step ld = cur;
  MG_LDS_POISON_STAGE(lds, NS * STAGE);
  // prologue: steps 0 .. NS-2
#pragma unroll
  for (int q = 0; q < NS - 1; ++q) {
    if (q < T) {
      issue(ld, q);
      advance(ld, a);
    }
  }
  for (int t = 0; t < T; ++t) {
    // step t landed when at most the later steps' DMAs are outstanding
    if (t + NS - 2 < T) wait_vmcnt<(NS - 2) * DPS>();
    else wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if (t + NS - 1 < T) {
      MG_LDS_POISON_STAGE(lds + ((t + NS - 1) % NS) * STAGE, STAGE);
      issue(ld, (t + NS - 1) % NS);
      advance(ld, a);
    }
    const unsigned char *As = lds + (t % NS) * STAGE;
    const unsigned char *Bs = As + BM * SB;
#pragma unroll
    for (int h = 0; h < SB / 64; ++h) {
      i4v fa[FMW], fb[FNW];
#pragma unroll
      for (int i = 0; i < FMW; ++i) {
        const int row = wm0 + 16 * i + l16;
        fa[i] = *reinterpret_cast<const i4v *>(As + row * SB + swz_chunk<SB>(row, h * 4 + g) * 16);
      }
#pragma unroll
      for (int j = 0; j < FNW; ++j) {
        const int row = wn0 + 16 * j + l16;
        fb[j] = *reinterpret_cast<const i4v *>(Bs + row * SB + swz_chunk<SB>(row, h * 4 + g) * 16);
      }
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j) acc[i][j] = M::mma(fa[i], fb[j], acc[i][j]);
    }
    const bool seg_last = cur.st + 1 == seg_len(cur.seg, a);
    if (CHUNK > 0 && ((cur.st + 1) % (CHUNK > 0 ? CHUNK : 1) == 0 || seg_last)) {
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dacc[i][j][r] += (int)acc[i][j][r];
            acc[i][j][r] = 0;
          }
    }
    if (t + 1 < T && seg_last && cur.p == pmax_of(cur.d, a.s))
      fold_partials<M, FMW, FNW, S::THREADS>(acc, dacc, plane, ldexp(1.0, -a.bits * cur.d),
                                             cur.seg == 0 && cur.d == 2);
    advance(cur, a);
  }

  // Last diagonal of the last segment, then the epilogue.
  const bool only = a.s == 1 && a.seg_stages >= a.total_stages;  // a single fold in all
  finish_tile<M, FMW, FNW, S::THREADS>(a, acc, dacc, plane, only, m0 + wm0 + 4 * g,
                                       n0 + wn0 + l16);
}

template <int ALGO, int WGM, int WGN, int FMW, int FNW, int NS, int SB>
__global__ __launch_bounds__((SplitDmaShape<WGM, WGN, FMW, FNW, NS, SB>::THREADS),
                             (SplitDmaShape<WGM, WGN, FMW, FNW, NS, SB>::MINW)) void
split_gemm_dma_kernel(SplitArgs a, int tiles_m, int tiles_n) {
  typedef SplitDmaShape<WGM, WGN, FMW, FNW, NS, SB> S;
  extern __shared__ __align__(16) unsigned char lds[];
  int tm, tn;
  grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  split_dma_tile<ALGO, WGM, WGN, FMW, FNW, NS, SB>(
      a, tm * S::BM, tn * S::BN, a.P + (int64_t)blockIdx.x * (S::BM * S::BN), lds);
}

// ---------------------------------------------------------------------------
// Pair-parallel division (for grids with fewer than one 128x128 tile per
// CU).  The s(s+1)/2 slice pairs, in the order the fused kernels walk them
// (d = 2..s+1, then p), are cut into G contiguous groups of near-equal
// size; workgroup (group g, tile) sums only its group's pairs and writes, for
// every diagonal d the group touches and every k segment, the exact INT32
// partial sum of P_d to a slot of Q (row-major [mp][np] per slot).  A second
// kernel adds a diagonal's partial sums (exact integers: the sum is P_d
// itself) and folds P_d 2^(-b d) into FP64 in increasing d with the same
// operations as the fused kernels' folds and epilogue, so the result is the
// same bit for bit; only the order in which the integer parts are formed
// differs, and integer addition is exact.
constexpr int kMaxPairGroups = 32;

struct PairGroups {
  int G, slots, nseg;
  int16_t pb[kMaxPairGroups], pe[kMaxPairGroups];   // pair range [pb, pe) of group g
  int16_t dlo[kMaxPairGroups], dhi[kMaxPairGroups]; // diagonals it touches
  int16_t base[kMaxPairGroups];                     // its first slot (for dlo)
};

// Pair index -> (d, p) in walk order, by stepping from (2, 1).
__device__ __forceinline__ void pair_of(int pi, int s, int &d, int &p) {
  d = 2;
  p = 1;
  for (int i = 0; i < pi; ++i) {
    if (++p > pmax_of(d, s)) {
      ++d;
      p = max(1, d - s);
    }
  }
}

template <int ALGO, int MINB>
__global__ __launch_bounds__(256, MINB) void split_pairs_kernel(SplitArgs a, PairGroups pg,
                                                                 int tiles_m, int tiles_n) {
  typedef SplitMma<ALGO> M;
  typedef typename M::acc_t Acc;
  typedef SplitShape<2, 2, 4, 4> S;  // 128x128 tile, 4 wavefronts of 64x64
  constexpr int FMW = 4, FNW = 4;
  constexpr int BM = S::BM, BN = S::BN, STAGE = S::STAGE;
  constexpr int CPR = kStageBytes / 16;
  extern __shared__ __align__(16) unsigned char lds[];

  const int tiles = tiles_m * tiles_n;
  const int grp = blockIdx.x / tiles, tb = blockIdx.x % tiles;
  int tm, tn;
  grouped_tile(tb, tiles_m, tiles_n, 8, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / 2) * 16 * FMW, wn0 = (wave % 2) * 16 * FNW;
  const int g = lane >> 4, l16 = lane & 15;

  const int64_t a_slice = (int64_t)a.mp * a.kp_bytes, b_slice = (int64_t)a.np * a.kp_bytes;
  int arow[S::NA], acol[S::NA], brow[S::NB], bcol[S::NB];
#pragma unroll
  for (int u = 0; u < S::NA; ++u) {
    const int q = tid + S::THREADS * u;
    arow[u] = q / CPR;
    acol[u] = (q % CPR) * 16;
  }
#pragma unroll
  for (int u = 0; u < S::NB; ++u) {
    const int q = tid + S::THREADS * u;
    brow[u] = q / CPR;
    bcol[u] = (q % CPR) * 16;
  }
  const unsigned char *abase = a.As + (int64_t)m0 * a.kp_bytes;
  const unsigned char *bbase = a.Bs + (int64_t)n0 * a.kp_bytes;

  // the group's walk: for each segment, pairs pb .. pe-1, each over the
  // segment's stages
  struct GStep {
    int seg, pi, d, p, st;
  };
  const int pb = pg.pb[grp], pe = pg.pe[grp];
  GStep first;
  first.seg = 0;
  first.pi = pb;
  first.st = 0;
  pair_of(pb, a.s, first.d, first.p);
  auto advance_g = [&](GStep &x) {
    if (++x.st < seg_len(x.seg, a)) return;
    x.st = 0;
    if (++x.pi < pe) {
      if (++x.p > pmax_of(x.d, a.s)) {
        ++x.d;
        x.p = max(1, x.d - a.s);
      }
      return;
    }
    ++x.seg;
    x.pi = pb;
    x.d = first.d;
    x.p = first.p;
  };

  i4v ra[S::NA], rb[S::NB];
  auto load = [&](const GStep &x) {
    const int64_t koff = (int64_t)(x.seg * a.seg_stages + x.st) * kStageBytes;
    const unsigned char *pa = abase + (x.p - 1) * a_slice + koff;
    const unsigned char *pbp = bbase + (x.d - x.p - 1) * b_slice + koff;
#pragma unroll
    for (int u = 0; u < S::NA; ++u)
      ra[u] = *reinterpret_cast<const i4v *>(pa + arow[u] * a.kp_bytes + acol[u]);
#pragma unroll
    for (int u = 0; u < S::NB; ++u)
      rb[u] = *reinterpret_cast<const i4v *>(pbp + brow[u] * a.kp_bytes + bcol[u]);
  };
  auto store = [&](int stage) {
    unsigned char *As = lds + stage * STAGE;
    unsigned char *Bs = As + BM * kPitch;
#pragma unroll
    for (int u = 0; u < S::NA; ++u)
      *reinterpret_cast<i4v *>(As + arow[u] * kPitch + acol[u]) = ra[u];
#pragma unroll
    for (int u = 0; u < S::NB; ++u)
      *reinterpret_cast<i4v *>(Bs + brow[u] * kPitch + bcol[u]) = rb[u];
  };

  Acc acc[FMW][FNW];
  i4v dacc[FMW][FNW];
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j = 0; j < FNW; ++j) {
      acc[i][j] = Acc{};
      dacc[i][j] = i4v{};
    }
  const int64_t plane = (int64_t)a.mp * a.np;
  const int row0 = m0 + wm0 + 4 * g, col0 = n0 + wn0 + l16;

  const int T = (pe - pb) * a.total_stages;
  GStep cur = first;
  MG_LDS_POISON_STAGE(lds, 2 * STAGE);
  load(cur);
  store(0);
  __syncthreads();
  for (int t = 0; t < T; ++t) {
    MG_LDS_POISON_STAGE(lds + ((t + 1) & 1) * STAGE, STAGE);
    GStep nxt = cur;
    advance_g(nxt);
    if (t + 1 < T) load(nxt);
    const unsigned char *As = lds + (t & 1) * STAGE;
    const unsigned char *Bs = As + BM * kPitch;
#pragma unroll
    for (int h = 0; h < kStageBytes / 64; ++h) {
      i4v fa[FMW], fb[FNW];
#pragma unroll
      for (int i = 0; i < FMW; ++i)
        fa[i] = *reinterpret_cast<const i4v *>(As + (wm0 + 16 * i + l16) * kPitch + h * 64 + g * 16);
#pragma unroll
      for (int j = 0; j < FNW; ++j)
        fb[j] = *reinterpret_cast<const i4v *>(Bs + (wn0 + 16 * j + l16) * kPitch + h * 64 + g * 16);
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j) acc[i][j] = M::mma(fa[i], fb[j], acc[i][j]);
    }
    const bool seg_last = cur.st + 1 == seg_len(cur.seg, a);
    if (M::CHUNK_STAGES > 0 && ((cur.st + 1) % (M::CHUNK_STAGES > 0 ? M::CHUNK_STAGES : 1) == 0 ||
                                seg_last)) {
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dacc[i][j][r] += (int)acc[i][j][r];
            acc[i][j][r] = 0;
          }
    }
    // last pair of its diagonal within this group (and segment): write the
    // group's part of P_d for this segment, then start the next diagonal
    const bool diag_end = seg_last && (cur.pi + 1 == pe || cur.p == pmax_of(cur.d, a.s));
    if (diag_end) {
      int32_t *q = a.Q + ((int64_t)cur.seg * pg.slots + pg.base[grp] + (cur.d - pg.dlo[grp])) * plane;
#pragma unroll
      for (int i = 0; i < FMW; ++i)
#pragma unroll
        for (int j = 0; j < FNW; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int v = M::CHUNK_STAGES > 0 ? dacc[i][j][r] : (int)acc[i][j][r];
            q[(int64_t)(row0 + 16 * i + r) * a.np + col0 + 16 * j] = v;
            dacc[i][j][r] = 0;
            if (M::CHUNK_STAGES == 0) acc[i][j][r] = 0;
          }
    }
    if (t + 1 < T) store((t + 1) & 1);
    __syncthreads();
    cur = nxt;
  }
}

// C <- alpha * 2^(E_i+F_j) * sum_d P_d 2^(-b d) + beta * C from the partial
// diagonal sums of split_pairs_kernel: per output, P_d of each segment is the
// exact sum of the groups' parts, folded in the fused kernels' order
// (segments, then increasing d; the first fold starts from 0) with the same
// fused multiply-adds and the same epilogue arithmetic.
__global__ void split_fold_kernel(SplitArgs a, PairGroups pg) {
  const int64_t total = (int64_t)a.m * a.n;
  const int64_t plane = (int64_t)a.mp * a.np;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / a.n), col = (int)(e % a.n);
    const int64_t at = (int64_t)row * a.np + col;
    double part = 0.0, fin = 0.0;
    bool first = true;
    for (int seg = 0; seg < pg.nseg; ++seg)
      for (int d = 2; d <= a.s + 1; ++d) {
        long long v = 0;
        for (int gq = 0; gq < pg.G; ++gq)
          if (pg.dlo[gq] <= d && d <= pg.dhi[gq])
            v += a.Q[((int64_t)seg * pg.slots + pg.base[gq] + (d - pg.dlo[gq])) * plane + at];
        const double sc = ldexp(1.0, -a.bits * d);
        if (seg == pg.nseg - 1 && d == a.s + 1) {
          fin = fma((double)(int)v, sc, first ? 0.0 : part);
        } else {
          part = fma((double)(int)v, sc, first ? 0.0 : part);
          first = false;
        }
      }
    const double prod = ldexp(fin, a.E[row] + a.F[col]);
    double *c = a.C + (int64_t)row * a.ldc + col;
    double o = __dmul_rn(a.alpha, prod);
    if (a.beta != 0.0) o = __dadd_rn(o, __dmul_rn(a.beta, *c));
    *c = o;
  }
}

template <typename K>
int ensure_lds(K kern, size_t bytes) {
  MG_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return MG_OK;
}

template <int ALGO, int WGM, int WGN, int FMW, int FNW>
int launch_split_t(const SplitArgs &a, const SplitLayout &L, hipStream_t s) {
  typedef SplitShape<WGM, WGN, FMW, FNW> S;
  // Register budget: INT8 accumulators fit two 4-wavefront workgroups per CU
  // for the 128x128 tiles; bigger tiles and BF16 run one per CU.
  constexpr int MINB = (ALGO == MG_SPLIT_I8 && FMW * FNW <= 16) ? 2 : 1;
  auto kern = split_gemm_kernel<ALGO, WGM, WGN, FMW, FNW, MINB>;
  static int once = ensure_lds(kern, S::LDS_BYTES);
  if (once != MG_OK) return once;
  const int tiles_m = (int)(L.mp / S::BM), tiles_n = (int)(L.np / S::BN);
  hipLaunchKernelGGL(kern, dim3(tiles_m * tiles_n), dim3(S::THREADS), S::LDS_BYTES, s, a, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <int ALGO, int WGM, int WGN, int FMW, int FNW, int NS, int SB>
int launch_split_dma_t(const SplitArgs &a128, const SplitLayout &L, hipStream_t s) {
  typedef SplitDmaShape<WGM, WGN, FMW, FNW, NS, SB> S;
  auto kern = split_gemm_dma_kernel<ALGO, WGM, WGN, FMW, FNW, NS, SB>;
  static int once = ensure_lds(kern, S::LDS_BYTES);
  if (once != MG_OK) return once;
  SplitArgs a = a128;  // stage counts in SB-byte stages
  a.total_stages = a128.total_stages * (kStageBytes / SB);
  a.seg_stages = a128.seg_stages * (kStageBytes / SB);
  const int tiles_m = (int)(L.mp / S::BM), tiles_n = (int)(L.np / S::BN);
  hipLaunchKernelGGL(kern, dim3(tiles_m * tiles_n), dim3(S::THREADS), S::LDS_BYTES, s, a, tiles_m,
                     tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <int WGM, int WGN, int FMW, int FNW, int NS, int SB = 128>
int launch_split_dma(int algo, const SplitArgs &a, const SplitLayout &L, hipStream_t s) {
  return algo == MG_SPLIT_BF16
             ? launch_split_dma_t<MG_SPLIT_BF16, WGM, WGN, FMW, FNW, NS, SB>(a, L, s)
             : launch_split_dma_t<MG_SPLIT_I8, WGM, WGN, FMW, FNW, NS, SB>(a, L, s);
}

template <int ALGO>
int launch_pairs(const SplitArgs &a, const PairGroups &pg, const SplitLayout &L, hipStream_t s) {
  typedef SplitShape<2, 2, 4, 4> S;
  constexpr int MINB = ALGO == MG_SPLIT_I8 ? 2 : 1;  // as the fused 128x128 register tile
  auto kern = split_pairs_kernel<ALGO, MINB>;
  static int once = ensure_lds(kern, S::LDS_BYTES);
  if (once != MG_OK) return once;
  const int tiles_m = (int)(L.mp / S::BM), tiles_n = (int)(L.np / S::BN);
  hipLaunchKernelGGL(kern, dim3((unsigned)(tiles_m * tiles_n * pg.G)), dim3(S::THREADS),
                     S::LDS_BYTES, s, a, pg, tiles_m, tiles_n);
  MG_HIP_TRY(hipGetLastError());
  const int64_t total = (int64_t)a.m * a.n;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 4096);
  hipLaunchKernelGGL(split_fold_kernel, dim3(blocks), dim3(256), 0, s, a, pg);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

template <int WGM, int WGN, int FMW, int FNW>
int launch_split(int algo, const SplitArgs &a, const SplitLayout &L, hipStream_t s) {
  return algo == MG_SPLIT_BF16 ? launch_split_t<MG_SPLIT_BF16, WGM, WGN, FMW, FNW>(a, L, s)
                               : launch_split_t<MG_SPLIT_I8, WGM, WGN, FMW, FNW>(a, L, s);
}

// ---------------------------------------------------------------------------
// Batched split GEMM: many independent problems in one set of launches, at
// the default slice count.  The preparation launches run one grid over the
// blocks of all problems (a workgroup finds its problem by binary search over
// the block prefix sums); the product launch runs one workgroup per 64x64
// output tile of every problem, longest k first, with the all-pairs tile
// below -- the same slices, exact integer diagonal sums and FP64 folds in the
// same order as the single-problem divisions, so each result is the one a
// single call gives, bit for bit.  Per problem the workspace holds only what
// those tiles read: E and F, and slices of A and B padded to 64 rows /
// columns and 128 k.
struct SplitPrepDesc {
  const double *A, *B;
  int64_t lda, ldb, kp;
  int m, n, k, mp, np;
  int nr;      // columns of B the product tiles read: n rounded up to the tile
  int cx, cy;  // column-exponent blocks: cx blocks of 256 columns x cy k-chunk strides
  int rpb;     // rows of A per block: 16, 8, 4 (4, 2, 1 per wavefront; kp <= 256, 512,
               // 1024) or 1
  int *E, *F;
  unsigned char *As, *Bs;
};

struct SplitTileRec {
  int prob, m0, n0, pad;
};

constexpr int kBatchTile = 64;  // output tile of the batched product (64x64)

// Problem that owns block b of a batched launch: the last i with first[i] <= b.
__device__ __forceinline__ int batch_problem(const int *first, int count, int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void batched_fill_kernel(const SplitPrepDesc *d,
                                                           const int *first, int count) {
  const int i = batch_problem(first, count, blockIdx.x);
  fill_int_body(d[i].F, d[i].nr, INT_MIN, blockIdx.x - first[i]);
}

// Blocks [0, cx*cy) of a problem find column exponents of B; each further
// block finds the exponent of one row of A and slices it.
template <int ESZ>
__global__ __launch_bounds__(256) void batched_exp_rows_kernel(const SplitPrepDesc *d,
                                                               const int *first, int count,
                                                               int s, int bits) {
  const int i = batch_problem(first, count, blockIdx.x);
  const SplitPrepDesc &q = d[i];
  const int lb = blockIdx.x - first[i], ncol = q.cx * q.cy;
  if (lb < ncol)
    col_exp_body(q.B, q.ldb, q.k, q.n, q.F, lb % q.cx, lb / q.cx, q.cy);
  else if (q.rpb == 1)
    slice_rows_exp_body<ESZ>(q.A, q.lda, q.m, q.k, q.mp, q.kp, q.E, s, bits, q.As, lb - ncol);
  else if (q.rpb == 16)
    slice_rows_wave_body<ESZ, 16>(q.A, q.lda, q.m, q.k, q.mp, q.kp, q.E, s, bits, q.As,
                                  (lb - ncol) * 16 + (int)(threadIdx.x >> 4));
  else if (q.rpb == 8)
    slice_rows_wave_body<ESZ, 32>(q.A, q.lda, q.m, q.k, q.mp, q.kp, q.E, s, bits, q.As,
                                  (lb - ncol) * 8 + (int)(threadIdx.x >> 5));
  else
    slice_rows_wave_body<ESZ, 64>(q.A, q.lda, q.m, q.k, q.mp, q.kp, q.E, s, bits, q.As,
                                  (lb - ncol) * 4 + (int)(threadIdx.x >> 6));
}

template <int ESZ>
__global__ __launch_bounds__(256) void batched_slice_cols_kernel(const SplitPrepDesc *d,
                                                                 const int *first, int count,
                                                                 int s, int bits) {
  const int i = batch_problem(first, count, blockIdx.x);
  const SplitPrepDesc &q = d[i];
  slice_cols_body<ESZ>(q.B, q.ldb, q.k, q.n, q.np, q.kp, q.F, s, bits, q.Bs,
                       blockIdx.x - first[i]);
}

// All-pairs tile: one 64x64 output tile on 4 wavefronts (32x32 each).  Per
// k stage of 64 bytes (64 INT8 / 32 BF16 values, one MFMA per 16x16 block)
// all S slices of A and all S slices of B for the tile are in LDS at once
// and every slice pair (p, q), p + q <= S + 1, is multiplied from them into
// one exact INT32 accumulator set per diagonal d = p + q, held in registers
// with the FP64 partial sums.  So each slice byte is read from memory once
// per tile (the pair-major walk reads slice p of A once for each of its
// S + 1 - p diagonals).  At the end of each k segment the diagonals fold in
// increasing d, the fold order of the other divisions: P_d of a segment is
// the same exact integer whatever order its pairs and stages are summed
// in, so the result is the same bit for bit.
// NS = 2: a 2-stage ring, one workgroup per CU; NS = 1: one stage, refilled
// after every workgroup has read it, two workgroups per CU (each one's loads
// and per-tile work overlap the other's products).
template <int S, int NS_ = 2>
struct AllPairsShape {
  static constexpr int THREADS = 256, BM = 64, BN = 64, SB = 64, NS = NS_, FMW = 2, FNW = 2;
  static constexpr int SLICE = 64 * SB;         // one slice's tile rows for one stage
  static constexpr int STAGE = 2 * S * SLICE;   // S slices of A, then S of B
  static constexpr size_t LDS_BYTES = (size_t)NS * STAGE;
  static_assert(LDS_BYTES <= 160 * 1024, "stage ring beyond the CU's LDS");
};

// Epilogue of an all-pairs tile: the last diagonal's integer sums, folded
// onto the partial sums, then C as in finish_tile.
template <int FMW, int FNW>
__device__ __forceinline__ void finish_ints(const SplitArgs &a, const i4v (&last)[FMW][FNW],
                                            const double (&part)[FMW][FNW][4], bool only,
                                            int row0, int col0) {
  const double sc = ldexp(1.0, -a.bits * (a.s + 1));
#pragma unroll
  for (int i = 0; i < FMW; ++i) {
    double fin[4][FNW];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < FNW; ++j)
        fin[r][j] = fma((double)last[i][j][r], sc, only ? 0.0 : part[i][j][r]);
    store_block<FNW>(a, fin, row0 + 16 * i, col0);
  }
}

// `a.seg_stages` and `a.total_stages` count 64-byte stages here; a.s == S.
template <int ALGO, int S, int NS>
__device__ __forceinline__ void split_allpairs_tile(const SplitArgs &a, int m0, int n0,
                                                    unsigned char *lds) {
  typedef AllPairsShape<S, NS> SH;
  constexpr int FMW = SH::FMW, FNW = SH::FNW, SB = SH::SB, SL = SH::SLICE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int g = lane >> 4, l16 = lane & 15;
  const int64_t a_slice = (int64_t)a.mp * a.kp_bytes, b_slice = (int64_t)a.np * a.kp_bytes;
  // DMA: wavefront w loads rows 16w .. 16w+15 of every slice (1 KB per
  // instruction); the lane supplies row 16w + lane/4, physical chunk lane%4,
  // which holds logical chunk swz_chunk(row, lane%4).
  const int drow = 16 * wave + (lane >> 2);
  const int64_t asrc = (int64_t)(m0 + drow) * a.kp_bytes + swz_chunk<SB>(drow, lane & 3) * 16;
  const int64_t bsrc = (int64_t)(n0 + drow) * a.kp_bytes + swz_chunk<SB>(drow, lane & 3) * 16;
  auto issue = [&](int st, int stage) {
    const int64_t koff = (int64_t)st * SB;
    unsigned char *la = lds + stage * SH::STAGE + wave * 1024;
#pragma unroll
    for (int t = 0; t < S; ++t) dma16(a.As + t * a_slice + asrc + koff, la + t * SL);
#pragma unroll
    for (int t = 0; t < S; ++t) dma16(a.Bs + t * b_slice + bsrc + koff, la + (S + t) * SL);
  };

  i4v acc[S][FMW][FNW];  // INT32 sums of the diagonals d = 2 .. S+1 (index d - 2)
  double part[FMW][FNW][4];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int i = 0; i < FMW; ++i)
#pragma unroll
      for (int j = 0; j < FNW; ++j) acc[d][i][j] = i4v{};
#pragma unroll
  for (int i = 0; i < FMW; ++i)
#pragma unroll
    for (int j = 0; j < FNW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[i][j][r] = 0.0;

  const int T = a.total_stages;
  bool first = true;  // no fold yet: the first starts from 0
  if constexpr (NS == 2) {
    MG_LDS_POISON_STAGE(lds, SH::NS * SH::STAGE);
    issue(0, 0);
  }
  for (int t = 0; t < T; ++t) {
    if constexpr (NS == 1) {
      MG_LDS_POISON_STAGE(lds, SH::STAGE);
      issue(t, 0);
    }
    wait_vmcnt<0>();
    __builtin_amdgcn_s_barrier();
    if constexpr (NS == 2) {
      if (t + 1 < T) {
        MG_LDS_POISON_STAGE(lds + ((t + 1) & 1) * SH::STAGE, SH::STAGE);
        issue(t + 1, (t + 1) & 1);
      }
    }
    const unsigned char *As = lds + (NS == 2 ? (t & 1) : 0) * SH::STAGE;
    const unsigned char *Bs = As + S * SL;
    i4v fb[S][FNW];
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int j = 0; j < FNW; ++j) {
        const int row = wn0 + 16 * j + l16;
        fb[q][j] = *reinterpret_cast<const i4v *>(Bs + q * SL + row * SB +
                                                  swz_chunk<SB>(row, g) * 16);
      }
#pragma unroll
    for (int p = 0; p < S; ++p) {
      i4v fa[FMW];
#pragma unroll
      for (int i = 0; i < FMW; ++i) {
        const int row = wm0 + 16 * i + l16;
        fa[i] = *reinterpret_cast<const i4v *>(As + p * SL + row * SB +
                                               swz_chunk<SB>(row, g) * 16);
      }
#pragma unroll
      for (int q = 0; q < S - p; ++q)
#pragma unroll
        for (int i = 0; i < FMW; ++i)
#pragma unroll
          for (int j = 0; j < FNW; ++j) {
            if constexpr (ALGO == MG_SPLIT_I8) {
              acc[p + q][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[i], fb[q][j],
                                                                       acc[p + q][i][j], 0, 0, 0);
            } else {  // 32 products of |x| <= 255^2: exact in FP32, then added as integers
              const f4v c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf8v, fa[i]), __builtin_bit_cast(bf8v, fb[q][j]), f4v{},
                  0, 0, 0);
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[p + q][i][j][r] += (int)c[r];
            }
          }
    }
    // one stage: every wavefront has read it before the next load overwrites it
    if constexpr (NS == 1) __builtin_amdgcn_s_barrier();
    // End of a k segment (but not the last): fold every diagonal, increasing d.
    if (t + 1 < T && (t + 1) % a.seg_stages == 0) {
#pragma unroll
      for (int d = 0; d < S; ++d) {
        const double sc = ldexp(1.0, -a.bits * (d + 2));
#pragma unroll
        for (int i = 0; i < FMW; ++i)
#pragma unroll
          for (int j = 0; j < FNW; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              part[i][j][r] = fma((double)acc[d][i][j][r], sc, first ? 0.0 : part[i][j][r]);
              acc[d][i][j][r] = 0;
            }
        first = false;
      }
    }
  }
  // Last segment: diagonals 2 .. S, then the last one in the epilogue.
#pragma unroll
  for (int d = 0; d < S - 1; ++d) {
    const double sc = ldexp(1.0, -a.bits * (d + 2));
#pragma unroll
    for (int i = 0; i < FMW; ++i)
#pragma unroll
      for (int j = 0; j < FNW; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[i][j][r] = fma((double)acc[d][i][j][r], sc, first ? 0.0 : part[i][j][r]);
    first = false;
  }
  finish_ints<FMW, FNW>(a, acc[S - 1], part, first, m0 + wm0 + 4 * g, n0 + wn0 + l16);
}

template <int ALGO, int S, int NS>
__global__ __launch_bounds__(256, NS == 1 ? 2 : 1) void split_allpairs_kernel(
    const SplitArgs *args, const SplitTileRec *recs) {
  extern __shared__ __align__(16) unsigned char lds[];
  const SplitTileRec r = recs[blockIdx.x];
  if (r.prob < 0) return;  // padding of an XCD's share of the list
  const SplitArgs a = args[r.prob];
  split_allpairs_tile<ALGO, S, NS>(a, r.m0, r.n0, lds);
}

// The all-pairs tile over one problem's 64x64 tiles (work division 16).
template <int ALGO, int S, int NS>
__global__ __launch_bounds__(256, NS == 1 ? 2 : 1) void split_allpairs_grid_kernel(
    SplitArgs a, int tiles_m, int tiles_n) {
  extern __shared__ __align__(16) unsigned char lds[];
  int tm, tn;
  grouped_tile(xcd_remap(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  split_allpairs_tile<ALGO, S, NS>(a, tm * 64, tn * 64, lds);
}

// Stages of the batched product tile: one, with two workgroups per CU
// (measured against the 2-stage ring at one per CU, 2000-problem batch:
// INT8 1.92 against 2.05 ms, BF16 2.53 against 3.01 ms; uniform 1024^3
// batches 0.70 against 0.91 ms).
constexpr int kAllPairsNS = 1;

// Slice count of a batch (the all-pairs tile is built for the default).
constexpr int batch_slices(int algo) { return algo == MG_SPLIT_BF16 ? 6 : 7; }

template <int ALGO>
int launch_batched_t(const SplitArgs *d_args, const SplitPrepDesc *d_desc, const int *d_first,
                     int nl, const int64_t *blocks, const SplitTileRec *d_recs, int ntiles,
                     hipStream_t s) {
  constexpr int ESZ = ALGO == MG_SPLIT_BF16 ? 2 : 1;
  constexpr int S = batch_slices(ALGO);
  const int bits = split_bits(ALGO);
  typedef AllPairsShape<S, kAllPairsNS> SH;
  static int once = ensure_lds(split_allpairs_kernel<ALGO, S, kAllPairsNS>, SH::LDS_BYTES);
  if (once != MG_OK) return once;
  hipLaunchKernelGGL(batched_fill_kernel, dim3((unsigned)blocks[0]), dim3(256), 0, s, d_desc,
                     d_first, nl);
  hipLaunchKernelGGL(batched_exp_rows_kernel<ESZ>, dim3((unsigned)blocks[1]), dim3(256), 0, s,
                     d_desc, d_first + (nl + 1), nl, S, bits);
  hipLaunchKernelGGL(batched_slice_cols_kernel<ESZ>, dim3((unsigned)blocks[2]), dim3(256), 0, s,
                     d_desc, d_first + 2 * (nl + 1), nl, S, bits);
  hipLaunchKernelGGL((split_allpairs_kernel<ALGO, S, kAllPairsNS>), dim3((unsigned)ntiles),
                     dim3(256), SH::LDS_BYTES, s, d_args, d_recs);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

// Work division 16: the all-pairs tile on the single-problem workspace (its
// slice pitches mp, np; the partial-sum region unused); only the tiles that
// hold outputs run.  `a` counts 128-byte stages.
template <int ALGO>
int launch_allpairs_t(const SplitArgs &a128, hipStream_t s) {
  constexpr int S = batch_slices(ALGO);
  typedef AllPairsShape<S, kAllPairsNS> SH;
  if (a128.s != S) {
    set_error("split work division 16 takes the default slice count (%d)", S);
    return MG_ERR_INVALID_ARG;
  }
  auto kern = split_allpairs_grid_kernel<ALGO, S, kAllPairsNS>;
  static int once = ensure_lds(kern, SH::LDS_BYTES);
  if (once != MG_OK) return once;
  SplitArgs a = a128;  // stage counts in 64-byte stages
  a.total_stages = a128.total_stages * (kStageBytes / SH::SB);
  a.seg_stages = a128.seg_stages * (kStageBytes / SH::SB);
  const int tiles_m = (int)ceil_div(a.m, SH::BM), tiles_n = (int)ceil_div(a.n, SH::BN);
  hipLaunchKernelGGL(kern, dim3((unsigned)(tiles_m * tiles_n)), dim3(SH::THREADS), SH::LDS_BYTES,
                     s, a, tiles_m, tiles_n);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

}  // namespace

int split_default_slices(int algo) { return algo == MG_SPLIT_BF16 ? 6 : 7; }

int split_bits(int algo) { return algo == MG_SPLIT_BF16 ? 8 : 7; }

namespace {

// Longest k segment (in 128-byte stages) whose diagonal sums stay exact in
// INT32: slices * kseg * (2^b - 1)^2 < 2^31; BF16 segments hold whole
// 256-long FP32 chunks.  0 if even one stage would overflow.
int64_t seg_stages_of(int algo, int slices) {
  const int bits = split_bits(algo);
  const int64_t smax = (int64_t)((1u << bits) - 1) * ((1u << bits) - 1);
  const int64_t kseg = ((int64_t)INT32_MAX / (slices * smax));
  const int64_t per_stage = kStageBytes / (algo == MG_SPLIT_BF16 ? 2 : 1);
  int64_t st = kseg / per_stage;
  if (algo == MG_SPLIT_BF16) st -= st % SplitMma<MG_SPLIT_BF16>::CHUNK_STAGES;
  return st;
}

// Tiles of 128x128 below which the pair-parallel division serves (one per
// CU on the 256 CUs of MI355X), and the workgroups it aims for.
constexpr int64_t kPairTilesBelow = 256;
constexpr int64_t kPairTargetWgs = 512;

bool pairs_eligible(int64_t mp, int64_t np) { return (mp / 128) * (np / 128) < kPairTilesBelow; }

// Pair groups of the pair-parallel division for a padded shape: G groups of
// near-equal contiguous pair ranges, enough to give about kPairTargetWgs
// workgroups; their diagonal spans, slot bases and the segment count.
PairGroups pair_groups(int algo, int slices, int64_t mp, int64_t np, int64_t kp) {
  PairGroups pg{};
  const int P = slices * (slices + 1) / 2;
  const int64_t tiles = (mp / 128) * (np / 128);
  pg.G = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)P, (int64_t)kMaxPairGroups,
                                                      ceil_div(kPairTargetWgs, tiles)}));
  auto d_of = [&](int pi) {
    int d = 2, p = 1;
    for (int i = 0; i < pi; ++i)
      if (++p > std::min(slices, d - 1)) {
        ++d;
        p = std::max(1, d - slices);
      }
    return d;
  };
  int slots = 0;
  for (int g = 0; g < pg.G; ++g) {
    pg.pb[g] = (int16_t)((int64_t)g * P / pg.G);
    pg.pe[g] = (int16_t)((int64_t)(g + 1) * P / pg.G);
    pg.dlo[g] = (int16_t)d_of(pg.pb[g]);
    pg.dhi[g] = (int16_t)d_of(pg.pe[g] - 1);
    pg.base[g] = (int16_t)slots;
    slots += pg.dhi[g] - pg.dlo[g] + 1;
  }
  pg.slots = slots;
  const int64_t total_stages = kp * (algo == MG_SPLIT_BF16 ? 2 : 1) / kStageBytes;
  const int64_t seg = std::max<int64_t>(1, std::min(seg_stages_of(algo, slices), total_stages));
  pg.nseg = (int)ceil_div(total_stages, seg);
  return pg;
}

}  // namespace

int split_layout(int algo, int slices, int64_t m, int64_t n, int64_t k, SplitLayout *L) {
  if (algo != MG_SPLIT_I8 && algo != MG_SPLIT_BF16) {
    set_error("not a split algorithm: %d", algo);
    return MG_ERR_INVALID_ARG;
  }
  if (slices < 1 || slices > kSplitMaxSlices) {
    set_error("slices must be in [1, %d], got %d", kSplitMaxSlices, slices);
    return MG_ERR_INVALID_ARG;
  }
  if (m < 0 || n < 0 || k < 0) {
    set_error("negative extent");
    return MG_ERR_INVALID_ARG;
  }
  L->mp = round_up(std::max<int64_t>(m, 1), kSplitTileMN);
  L->np = round_up(std::max<int64_t>(n, 1), kSplitTileMN);
  L->kp = round_up(std::max<int64_t>(k, 1), kSplitTileK);
  L->elem_bytes = algo == MG_SPLIT_BF16 ? 2 : 1;
  int64_t off = 0;
  L->e_off = off;
  off = round_up(off + 4 * L->mp, 256);
  L->f_off = off;
  off = round_up(off + 4 * L->np, 256);
  L->a_off = off;
  off = round_up(off + slices * L->mp * L->kp * L->elem_bytes, 256);
  L->b_off = off;
  off = round_up(off + slices * L->np * L->kp * L->elem_bytes, 256);
  L->p_off = off;
  // FP64 partial sums of the fused divisions, or (shapes the pair-parallel
  // division serves) the INT32 partial diagonal sums of its groups
  int64_t pbytes = 8 * L->mp * L->np;
  if (pairs_eligible(L->mp, L->np)) {
    const PairGroups pg = pair_groups(algo, slices, L->mp, L->np, L->kp);
    pbytes = std::max<int64_t>(pbytes, (int64_t)pg.nseg * pg.slots * L->mp * L->np * 4);
  }
  off = round_up(off + pbytes, 256);
  L->total = off;
  return MG_OK;
}

int split_prepare(int algo, int slices, int64_t m, int64_t n, int64_t k, const double *A,
                  int64_t lda, const double *B, int64_t ldb, void *ws, hipStream_t s) {
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  unsigned char *w = static_cast<unsigned char *>(ws);
  int *E = reinterpret_cast<int *>(w + L.e_off);
  int *F = reinterpret_cast<int *>(w + L.f_off);
  const int bits = split_bits(algo);
  const int mp = (int)L.mp, np = (int)L.np;

  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, s, F, np,
                     INT_MIN);
  MG_HIP_TRY(hipGetLastError());
  // column-exponent blocks of B (none when B is empty)
  const int64_t cx = n > 0 && k > 0 ? ceil_div(n, 256) : 0;
  const int64_t cy = n > 0 && k > 0 ? std::min<int64_t>(ceil_div(k, kColRows), 4096) : 0;

  unsigned char *As = w + L.a_off, *Bs = w + L.b_off;
  const int64_t cblocks = (L.np / 64) * (L.kp / 64);
  // one workgroup of 256 lanes per row / per 64 x 64 block; the dispatch's
  // work-item count is 32-bit
  if (cblocks * 256 > (int64_t)UINT32_MAX || (cx * cy + mp) * 256 > (int64_t)UINT32_MAX) {
    set_error("split operands too large for one dispatch");
    return MG_ERR_INVALID_ARG;
  }
  if (algo == MG_SPLIT_BF16) {
    hipLaunchKernelGGL(exp_rows_kernel<2>, dim3((unsigned)(cx * cy + mp)), dim3(256), 0, s, A,
                       lda, (int)m, (int)k, mp, L.kp, E, slices, bits, As, B, ldb, (int)n, F,
                       (int)cx, (int)cy);
    hipLaunchKernelGGL(slice_cols_kernel<2>, dim3((unsigned)cblocks), dim3(256), 0, s, B, ldb,
                       (int)k, (int)n, np, L.kp, F, slices, bits, Bs);
  } else {
    hipLaunchKernelGGL(exp_rows_kernel<1>, dim3((unsigned)(cx * cy + mp)), dim3(256), 0, s, A,
                       lda, (int)m, (int)k, mp, L.kp, E, slices, bits, As, B, ldb, (int)n, F,
                       (int)cx, (int)cy);
    hipLaunchKernelGGL(slice_cols_kernel<1>, dim3((unsigned)cblocks), dim3(256), 0, s, B, ldb,
                       (int)k, (int)n, np, L.kp, F, slices, bits, Bs);
  }
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

int split_num_cfgs() { return 17; }

// Product-kernel work division (measured on MI355X at n = 4096): the 256x256
// direct-to-LDS tile once every CU gets one, then the 128x256 one, else the
// register-staged 128x128 tile.
int split_pick_cfg(int algo, int slices, int64_t mp, int64_t np, bool latency) {
  // For one call's latency, at the default slice count, the all-pairs 64x64
  // tile (16): INT8 at every size, BF16 up to n = 1024.  Whole INT8 call n =
  // 256 / 512 / 1024: 50 / 57 / 90 us against 76 / 100 / 139 for the
  // pair-parallel division and the 128x128 ring; products with a held
  // workspace, n = 2048 / 3072 / 4096 / 5120 / 6144 / 8192: 0.21 / 0.73 /
  // 1.61 / 3.17 / 5.52 / 11.99 ms against 0.23 / 1.57 / 1.78 / 4.20 / 7.33 /
  // 12.69 for the 256x256 ring (whose tiles fill the chip only at n = 4096
  // and 8192).  BF16 n = 1024: 163 against 223 us; n = 2048 / 3072 about
  // even, n = 4096 4.24 against 3.19 ms (its FP32-to-INT32 conversions).
  if (latency && slices == split_default_slices(algo) &&
      (algo == MG_SPLIT_I8 || mp * np <= (int64_t)1024 * 1024))
    return 16;
  // Other slice counts below one 128x128 tile per CU: the pair-parallel
  // division (15): the fused divisions would give too few workgroups, each
  // walking all the slice pairs as one chain of dependent loads.  When the
  // device is shared (the server's batches) the fused divisions give more
  // throughput: same MFMA work without the partial sums' traffic.
  if (latency && pairs_eligible(mp, np)) return 15;
  // INT8: the 16-wave 256x256 tile once it fills the chip.  BF16 keeps its
  // FP32 chunk accumulators in registers: 128x128 tiles on 8 waves, two
  // workgroups per CU.  Below those, the 128x128 ring on 8 waves (whole
  // INT8 call, n = 512 / 1024 / 2048: 130 / 229 / 402 us against 190 / 342
  // / 573 for the register-staged 128x128 tile).
  if (algo == MG_SPLIT_I8 && (mp / 256) * (np / 256) >= 256) return 4;
  if (algo == MG_SPLIT_BF16) return 12;
  if ((mp / 128) * (np / 256) >= 256) return 2;
  // 3-stage ring below one 128x128 tile per CU, 2-stage (two workgroups per
  // CU) from there: alone / four streams at once, n = 1024: 228 / 72 us per
  // call (3 stages) against 226 / 85; n = 2048: 424 / 399 against 406 / 350
  return (mp / 128) * (np / 128) >= 256 ? 12 : 14;
}

int split_multiply(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                   double beta, double *C, int64_t ldc, void *ws, hipStream_t s, int cfg) {
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  unsigned char *w = static_cast<unsigned char *>(ws);
  SplitArgs a;
  a.P = reinterpret_cast<double *>(w + L.p_off);
  a.Q = nullptr;
  a.As = w + L.a_off;
  a.Bs = w + L.b_off;
  a.E = reinterpret_cast<const int *>(w + L.e_off);
  a.F = reinterpret_cast<const int *>(w + L.f_off);
  a.C = C;
  a.ldc = ldc;
  a.m = (int)m;
  a.n = (int)n;
  a.mp = (int)L.mp;
  a.np = (int)L.np;
  a.kp_bytes = L.kp * L.elem_bytes;
  a.s = slices;
  a.bits = split_bits(algo);
  a.total_stages = (int)(a.kp_bytes / kStageBytes);
  // Longest k segment whose diagonal sums stay exact in INT32:
  // slices * kseg * (2^b - 1)^2 < 2^31.
  const int64_t smax = (int64_t)((1u << a.bits) - 1) * ((1u << a.bits) - 1);
  const int64_t kseg = ((int64_t)INT32_MAX / (slices * smax));
  const int64_t per_stage = kStageBytes / L.elem_bytes;
  int64_t seg_stages = kseg / per_stage;
  if (algo == MG_SPLIT_BF16) seg_stages -= seg_stages % SplitMma<MG_SPLIT_BF16>::CHUNK_STAGES;
  if (seg_stages < 1) {
    set_error("too many slices for exact INT32 accumulation");
    return MG_ERR_INVALID_ARG;
  }
  a.seg_stages = (int)std::min<int64_t>(seg_stages, a.total_stages);
  a.alpha = alpha;
  a.beta = beta;
  if (cfg < 0) cfg = split_pick_cfg(algo, slices, L.mp, L.np, true);
  switch (cfg) {
    case 0: return launch_split<2, 2, 4, 4>(algo, a, L, s);          // 128x128, 4 waves, registers
    case 1: return launch_split_dma<2, 2, 4, 4, 4>(algo, a, L, s);   // 128x128, 4 waves, ring of 4
    case 2: return launch_split_dma<2, 4, 4, 4, 3>(algo, a, L, s);   // 128x256, 8 waves, ring of 3
    case 3: return launch_split_dma<2, 2, 8, 4, 3>(algo, a, L, s);   // 256x128, 4 waves, ring of 3
    case 4: return launch_split_dma<4, 4, 4, 4, 2>(algo, a, L, s);   // 256x256, 16 waves, ring of 2
    case 5: return launch_split_dma<2, 4, 4, 4, 2>(algo, a, L, s);   // 128x256, 8 waves, ring of 2
    case 6: return launch_split_dma<2, 4, 8, 4, 4, 64>(algo, a, L, s);  // 256x256, 8 waves, 4 x 64 B
    case 7: return launch_split_dma<4, 4, 4, 4, 4, 64>(algo, a, L, s);  // 256x256, 16 waves, 4 x 64 B
    case 8: return launch_split_dma<2, 4, 4, 4, 6, 64>(algo, a, L, s);  // 128x256, 8 waves, 6 x 64 B
    case 9: return launch_split_dma<2, 4, 8, 4, 4, 64>(algo, a, L, s);  // 256x256, 8 waves, 4 x 64 B
    case 10: return launch_split_dma<4, 2, 4, 8, 4, 64>(algo, a, L, s);  // 256x256, 8 waves, 4 x 64 B
    case 11: return launch_split_dma<2, 4, 8, 4, 2, 128>(algo, a, L, s);  // 256x256, 8 waves, 2 x 128 B
    case 12: return launch_split_dma<2, 4, 4, 2, 2, 128>(algo, a, L, s);  // 128x128, 8 waves, 2 x 128 B
    case 13: return launch_split_dma<2, 2, 4, 4, 2, 128>(algo, a, L, s);  // 128x128, 4 waves, 2 x 128 B
    case 14: return launch_split_dma<2, 4, 4, 2, 3, 128>(algo, a, L, s);  // 128x128, 8 waves, 3 x 128 B
    case 16:  // all-pairs 64x64 tile, one LDS stage, two workgroups per CU
      return algo == MG_SPLIT_BF16 ? launch_allpairs_t<MG_SPLIT_BF16>(a, s)
                                   : launch_allpairs_t<MG_SPLIT_I8>(a, s);
    case 15: {  // pair-parallel: groups of slice pairs x 128x128 tiles, then the fold
      if (!pairs_eligible(L.mp, L.np)) {
        set_error("split work division 15 serves shapes with fewer than %lld tiles of 128x128",
                  (long long)kPairTilesBelow);
        return MG_ERR_INVALID_ARG;
      }
      const PairGroups pg = pair_groups(algo, slices, L.mp, L.np, L.kp);
      a.Q = reinterpret_cast<int32_t *>(w + L.p_off);
      return algo == MG_SPLIT_BF16 ? launch_pairs<MG_SPLIT_BF16>(a, pg, L, s)
                                   : launch_pairs<MG_SPLIT_I8>(a, pg, L, s);
    }
  }
  set_error("unknown split cfg %d", cfg);
  return MG_ERR_INVALID_ARG;
}

int gemm_split(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
               double *C, int64_t ldc, void *ws, int64_t ws_bytes, hipStream_t s, int cfg) {
  if (m == 0 || n == 0) return MG_OK;
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  if (alpha == 0.0 || k == 0)  // C <- beta*C: A and B are not read
    return gemm_native(MG_F64, 0, m, n, 0, 0.0, nullptr, 1, nullptr, 1, beta, C, ldc, s);
  const int use = cfg < 0 ? split_pick_cfg(algo, slices, L.mp, L.np, true) : cfg;
  if (ws == nullptr || ws_bytes < split_ws_needed(L, use)) {
    set_error("split workspace too small: need %lld bytes", (long long)split_ws_needed(L, use));
    return MG_ERR_INVALID_ARG;
  }
  rc = split_prepare(algo, slices, m, n, k, A, lda, B, ldb, ws, s);
  if (rc != MG_OK) return rc;
  return split_multiply(algo, slices, m, n, k, alpha, beta, C, ldc, ws, s, cfg);
}

int64_t split_ws_needed(const SplitLayout &L, int cfg) {
  if (cfg == 16) return L.p_off;  // partial sums stay in registers
  return cfg == 15 ? L.total : round_up(L.p_off + 8 * L.mp * L.np, 256);
}

int64_t split_workspace_bytes(int algo, int slices, int64_t m, int64_t n, int64_t k,
                              bool latency) {
  SplitLayout L;
  if (split_layout(algo, slices, m, n, k, &L) != MG_OK) return -1;
  return split_ws_needed(L, split_pick_cfg(algo, slices, L.mp, L.np, latency));
}

namespace {

constexpr int kMaxPoolDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pools[kMaxPoolDevices] = {};

}  // namespace

// The library's stream-ordered pool for split workspaces on the current
// device: created on first use, it keeps freed blocks for reuse (no release
// threshold) instead of returning them to the device at every
// synchronization; mg_release_cached_memory trims it.  The caller's default
// pool is left as it is.
int workspace_pool(hipMemPool_t *out) {
  int dev = 0;
  MG_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxPoolDevices) {
    set_error("device %d beyond the %d the library supports", dev, kMaxPoolDevices);
    return MG_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pools[dev] == nullptr) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    MG_HIP_TRY(hipMemPoolCreate(&pool, &props));
    uint64_t thr = UINT64_MAX;
    const hipError_t e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    if (e != hipSuccess) {
      (void)hipMemPoolDestroy(pool);
      set_error("hipMemPoolSetAttribute failed: %s", hipGetErrorString(e));
      return MG_ERR_HIP;
    }
    g_pools[dev] = pool;
  }
  *out = g_pools[dev];
  return MG_OK;
}

int release_workspace_pools() {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (int d = 0; d < kMaxPoolDevices; ++d)
    if (g_pools[d] != nullptr) MG_HIP_TRY(hipMemPoolTrimTo(g_pools[d], 0));
  return MG_OK;
}

namespace {

// Stream-ordered workspace from the library's pool.
int pool_alloc(void **p, int64_t bytes, hipStream_t s) {
  hipMemPool_t pool = nullptr;
  int rc = workspace_pool(&pool);
  if (rc != MG_OK) return rc;
  const hipError_t e = hipMallocFromPoolAsync(p, (size_t)bytes, pool, s);
  if (e != hipSuccess) {
    set_error("workspace allocation (%lld bytes) failed: %s", (long long)bytes,
              hipGetErrorString(e));
    return MG_ERR_NO_MEMORY;
  }
  return MG_OK;
}

}  // namespace

int gemm_split_pooled(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                      double *C, int64_t ldc, hipStream_t s, bool latency) {
  if (m == 0 || n == 0) return MG_OK;
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  if (alpha == 0.0 || k == 0)
    return gemm_split(algo, slices, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, 0, s);
  const int cfg = split_pick_cfg(algo, slices, L.mp, L.np, latency);
  const int64_t bytes = split_ws_needed(L, cfg);
  void *ws = nullptr;
  rc = pool_alloc(&ws, bytes, s);
  if (rc != MG_OK) return rc;
  rc = gemm_split(algo, slices, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, ws, bytes, s, cfg);
  MG_HIP_TRY(hipFreeAsync(ws, s));
  return rc;
}

namespace {

// Host copies of batched-launch descriptors, each released once its stream
// has passed the copy that reads it.
std::mutex g_hold_mu;
std::vector<std::pair<std::vector<unsigned char> *, hipEvent_t>> g_hold;

void reap_holds() {
  std::lock_guard<std::mutex> lk(g_hold_mu);
  std::vector<std::pair<std::vector<unsigned char> *, hipEvent_t>> keep;
  for (auto &h : g_hold) {
    if (hipEventQuery(h.second) == hipSuccess) {
      delete h.first;
      (void)hipEventDestroy(h.second);
    } else {
      keep.push_back(h);
    }
  }
  g_hold.swap(keep);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int SplitBatchBuffers::reserve(size_t dev_bytes, size_t host_bytes) {
  // the caller guarantees that no launch still uses the old buffers
  // (doubling growth: a few reallocations over a server's life)
  if (dev_bytes > d_cap) {
    const size_t cap = std::max(dev_bytes, 2 * d_cap);
    if (d) (void)hipFree(d);
    d = nullptr;
    d_cap = 0;
    MG_HIP_TRY(hipMalloc(&d, cap));
    d_cap = cap;
  }
  if (host_bytes > h_cap) {
    const size_t cap = std::max({host_bytes, 2 * h_cap, (size_t)1 << 20});
    if (h) (void)hipHostFree(h);
    h = nullptr;
    h_cap = 0;
    MG_HIP_TRY(hipHostMalloc(&h, cap, hipHostMallocDefault));
    h_cap = cap;
  }
  return MG_OK;
}

void SplitBatchBuffers::release() {
  if (d) (void)hipFree(d);
  if (h) (void)hipHostFree(h);
  d = h = nullptr;
  d_cap = h_cap = 0;
}

// Rows of A per preparation block of the batched path (256 lanes): short
// rows share a wavefront (16 lanes per row up to 256 k, 32 up to 512, 64 up
// to 1024); longer rows take a whole block each.
static int64_t rows_per_block(int64_t kp) {
  return kp <= 256 ? 16 : kp <= 512 ? 8 : kp <= 1024 ? 4 : 1;
}

int gemm_split_batched(int algo, int64_t count, const mg_problem *probs, hipStream_t s,
                       SplitBatchBuffers *buf) {
  if (algo != MG_SPLIT_I8 && algo != MG_SPLIT_BF16) {
    set_error("not a split algorithm: %d", algo);
    return MG_ERR_INVALID_ARG;
  }
  reap_holds();
  const int slices = batch_slices(algo);
  const int64_t seg = seg_stages_of(algo, slices);
  if (seg < 1) {
    set_error("too many slices for exact INT32 accumulation");
    return MG_ERR_INVALID_ARG;
  }
  constexpr int64_t TILE = kBatchTile;
  // Degenerate problems as a single call runs them; the rest are batched.
  std::vector<int64_t> live;
  for (int64_t i = 0; i < count; ++i) {
    const mg_problem &q = probs[i];
    if (q.m == 0 || q.n == 0) continue;
    if (q.alpha == 0.0 || q.k == 0) {  // C <- beta*C: A and B are not read
      const int rc = gemm_native(MG_F64, 0, q.m, q.n, 0, 0.0, nullptr, 1, nullptr, 1, q.beta,
                                 q.C, q.ldc, s);
      if (rc != MG_OK) return rc;
      continue;
    }
    live.push_back(i);
  }
  const int nl = (int)live.size();
  if (nl == 0) return MG_OK;
  if (live.size() > (size_t)(INT32_MAX / 4)) {
    set_error("too many problems in one batch");
    return MG_ERR_INVALID_ARG;
  }
  // Per-problem workspace: E [mr], F [nr], A slices [s][mr][kp], B slices
  // [s][nr][kp] (B transposed), mr / nr = m / n rounded up to the tile.
  struct BLayout {
    int64_t mr, nr, kp, e_off, f_off, a_off, b_off;
  };
  const int64_t esz = algo == MG_SPLIT_BF16 ? 2 : 1;
  std::vector<BLayout> L((size_t)nl);
  std::vector<int64_t> woff((size_t)nl);
  int64_t wbytes = 0;
  for (int j = 0; j < nl; ++j) {
    const mg_problem &q = probs[live[(size_t)j]];
    BLayout &l = L[(size_t)j];
    l.mr = round_up(q.m, TILE);
    l.nr = round_up(q.n, TILE);
    // k padded to the all-pairs tile's 64-byte stage (INT8: 64 k, BF16: 32 k,
    // rounded up to 64 k so that the preparation's 64 x 64 blocks tile it):
    // zero slices past k add nothing, so the bits are those of the single
    // call, which pads to 128.
    l.kp = round_up(q.k, (int64_t)64);
    int64_t off = 0;
    l.e_off = off;
    off = round_up(off + 4 * l.mr, 256);
    l.f_off = off;
    off = round_up(off + 4 * l.nr, 256);
    l.a_off = off;
    off = round_up(off + slices * l.mr * l.kp * esz, 256);
    l.b_off = off;
    off = round_up(off + slices * l.nr * l.kp * esz, 256);
    woff[(size_t)j] = wbytes;
    wbytes += off;
  }
  // Longest k first: the costliest tiles start first and the short ones
  // fill in behind them.
  std::vector<int> ord((size_t)nl);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return L[(size_t)x].kp > L[(size_t)y].kp; });

  // Descriptor block: args [nl], prep descriptors [nl], three block prefix
  // arrays [nl + 1], tile records.
  std::vector<SplitArgs> args((size_t)nl);
  std::vector<SplitPrepDesc> desc((size_t)nl);
  std::vector<int> first((size_t)3 * (nl + 1), 0);
  std::vector<SplitTileRec> recs;
  int64_t blocks[3] = {0, 0, 0};
  for (int j = 0; j < nl; ++j) {
    const mg_problem &q = probs[live[(size_t)j]];
    const BLayout &l = L[(size_t)j];
    const int64_t nchunks = ceil_div(q.k, kColRows);
    const int64_t cx = ceil_div(q.n, 256), cy = std::min<int64_t>(nchunks, 256);
    const int64_t rpb = rows_per_block(l.kp);
    const int64_t nb[3] = {ceil_div(l.nr, 256), cx * cy + l.mr / rpb, (l.nr / 64) * (l.kp / 64)};
    for (int w = 0; w < 3; ++w) {
      first[(size_t)w * (nl + 1) + j] = (int)blocks[w];
      blocks[w] += nb[w];
      if (blocks[w] * 256 > (int64_t)UINT32_MAX) {
        set_error("split batch too large for one dispatch");
        return MG_ERR_INVALID_ARG;
      }
    }
  }
  for (int w = 0; w < 3; ++w) first[(size_t)w * (nl + 1) + nl] = (int)blocks[w];
  // Problems go to XCDs whole (the dispatcher places workgroup b on XCD
  // b mod 8), so the tiles that share a problem's slices share one L2:
  // problems, longest k first, each to the XCD with the least work so far.
  // A problem of 16 tiles or more is cut into 8 runs of consecutive tiles
  // (row-major, so a run shares rows of A), one per XCD, least loaded first.
  // The XCD lists are then interleaved, shorter ones padded with no-op
  // records.
  {
    constexpr int64_t kSpreadTiles = 16;
    std::vector<std::vector<SplitTileRec>> xl(kNumXcd);
    std::vector<double> load(kNumXcd, 0.0);
    std::vector<int> byload(kNumXcd);
    for (int j : ord) {
      const BLayout &l = L[(size_t)j];
      const int64_t tm = l.mr / TILE, tn = l.nr / TILE, nt = tm * tn;
      auto rec = [&](int64_t t) {
        return SplitTileRec{j, (int)((t / tn) * TILE), (int)((t % tn) * TILE), 0};
      };
      if (nt < kSpreadTiles) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[(size_t)x] += (double)nt * (double)l.kp;
        for (int64_t t = 0; t < nt; ++t) xl[(size_t)x].push_back(rec(t));
        continue;
      }
      std::iota(byload.begin(), byload.end(), 0);
      std::stable_sort(byload.begin(), byload.end(),
                       [&](int p, int q) { return load[(size_t)p] < load[(size_t)q]; });
      for (int c = 0; c < kNumXcd; ++c) {
        const int64_t t0 = nt * c / kNumXcd, t1 = nt * (c + 1) / kNumXcd;
        const int x = byload[(size_t)c];
        load[(size_t)x] += (double)(t1 - t0) * (double)l.kp;
        for (int64_t t = t0; t < t1; ++t) xl[(size_t)x].push_back(rec(t));
      }
    }
    size_t len = 0;
    for (const auto &v : xl) len = std::max(len, v.size());
    recs.assign(len * kNumXcd, SplitTileRec{-1, 0, 0, 0});
    for (int x = 0; x < kNumXcd; ++x)
      for (size_t i = 0; i < xl[(size_t)x].size(); ++i) recs[i * kNumXcd + (size_t)x] = xl[(size_t)x][i];
  }
  if (recs.size() * 256 > (size_t)UINT32_MAX) {
    set_error("split batch too large for one dispatch");
    return MG_ERR_INVALID_ARG;
  }
  const size_t o_args = 0;
  const size_t o_desc = align256(o_args + args.size() * sizeof(SplitArgs));
  const size_t o_first = align256(o_desc + desc.size() * sizeof(SplitPrepDesc));
  const size_t o_recs = align256(o_first + first.size() * sizeof(int));
  const size_t meta = align256(o_recs + recs.size() * sizeof(SplitTileRec));

  // Device memory: the caller's buffers (grown on demand), else the pool.
  void *dev = nullptr;
  int rc = MG_OK;
  if (buf != nullptr) {
    rc = buf->reserve((size_t)wbytes + meta, meta);
    if (rc != MG_OK) return rc;
    dev = buf->d;
  } else {
    rc = pool_alloc(&dev, wbytes + (int64_t)meta, s);
    if (rc != MG_OK) return rc;
  }
  unsigned char *w = static_cast<unsigned char *>(dev);
  const int bits = split_bits(algo);
  for (int j = 0; j < nl; ++j) {
    const mg_problem &q = probs[live[(size_t)j]];
    const BLayout &l = L[(size_t)j];
    unsigned char *base = w + woff[(size_t)j];
    SplitArgs &a = args[(size_t)j];
    a.P = nullptr;  // partial sums stay in registers
    a.Q = nullptr;
    a.As = base + l.a_off;
    a.Bs = base + l.b_off;
    a.E = reinterpret_cast<const int *>(base + l.e_off);
    a.F = reinterpret_cast<const int *>(base + l.f_off);
    a.C = static_cast<double *>(q.C);
    a.ldc = q.ldc;
    a.m = (int)q.m;
    a.n = (int)q.n;
    a.mp = (int)l.mr;  // slice pitches
    a.np = (int)l.nr;
    a.kp_bytes = l.kp * esz;
    a.s = slices;
    a.bits = bits;
    // stage counts in the all-pairs tile's 64-byte stages
    a.total_stages = (int)(a.kp_bytes / 64);
    a.seg_stages = (int)std::min<int64_t>(seg * (kStageBytes / 64), a.total_stages);
    a.alpha = q.alpha;
    a.beta = q.beta;
    SplitPrepDesc &d = desc[(size_t)j];
    d.A = static_cast<const double *>(q.A);
    d.B = static_cast<const double *>(q.B);
    d.lda = q.lda;
    d.ldb = q.ldb;
    d.kp = l.kp;
    d.m = (int)q.m;
    d.n = (int)q.n;
    d.k = (int)q.k;
    d.mp = (int)l.mr;
    d.np = (int)l.nr;
    d.nr = (int)l.nr;
    d.cx = (int)ceil_div(q.n, 256);
    d.cy = (int)std::min<int64_t>(ceil_div(q.k, kColRows), 256);
    d.rpb = (int)rows_per_block(l.kp);
    d.E = reinterpret_cast<int *>(base + l.e_off);
    d.F = reinterpret_cast<int *>(base + l.f_off);
    d.As = base + l.a_off;
    d.Bs = base + l.b_off;
  }
  // Host staging: the caller's pinned buffer, else a heap copy kept until
  // the stream has passed the copy.
  std::vector<unsigned char> *host = buf ? nullptr : new std::vector<unsigned char>(meta, 0);
  unsigned char *h = buf ? static_cast<unsigned char *>(buf->h) : host->data();
  std::memcpy(h + o_args, args.data(), args.size() * sizeof(SplitArgs));
  std::memcpy(h + o_desc, desc.data(), desc.size() * sizeof(SplitPrepDesc));
  std::memcpy(h + o_first, first.data(), first.size() * sizeof(int));
  std::memcpy(h + o_recs, recs.data(), recs.size() * sizeof(SplitTileRec));
  unsigned char *dm = w + wbytes;
  hipError_t e = hipMemcpyAsync(dm, h, meta, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    set_error("hipMemcpyAsync failed: %s", hipGetErrorString(e));
    rc = MG_ERR_HIP;
  }
  if (rc == MG_OK) {
    const auto *d_args = reinterpret_cast<const SplitArgs *>(dm + o_args);
    const auto *d_desc = reinterpret_cast<const SplitPrepDesc *>(dm + o_desc);
    const auto *d_first = reinterpret_cast<const int *>(dm + o_first);
    const auto *d_recs = reinterpret_cast<const SplitTileRec *>(dm + o_recs);
    rc = algo == MG_SPLIT_BF16
             ? launch_batched_t<MG_SPLIT_BF16>(d_args, d_desc, d_first, nl, blocks, d_recs,
                                               (int)recs.size(), s)
             : launch_batched_t<MG_SPLIT_I8>(d_args, d_desc, d_first, nl, blocks, d_recs,
                                             (int)recs.size(), s);
  }
  if (buf != nullptr) return rc;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess &&
      hipEventRecord(ev, s) == hipSuccess) {
    std::lock_guard<std::mutex> lk(g_hold_mu);
    g_hold.emplace_back(host, ev);
  } else {  // cannot tell when the copy is done: wait for it
    (void)hipStreamSynchronize(s);
    if (ev) (void)hipEventDestroy(ev);
    delete host;
  }
  e = hipFreeAsync(dev, s);
  if (rc == MG_OK && e != hipSuccess) {
    set_error("hipFreeAsync failed: %s", hipGetErrorString(e));
    rc = MG_ERR_HIP;
  }
  return rc;
}

}  // namespace mg
