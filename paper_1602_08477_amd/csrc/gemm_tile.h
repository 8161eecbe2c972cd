// One macro-tile of C <- alpha*A*B + beta*C on gfx950 matrix cores.
//
// This is the hierarchical tiling of the paper's single-source DGEMM
// (Section 4.2.2, Fig. 7): a block (workgroup) owns one tile of C, its
// threads stage tiles of A and B in shared memory (LDS), every thread
// accumulates a set of elements, and the block then moves on to the next
// A/B tiles along k.  Mapped to CDNA4:
//   grid    -> one dispatch (or a persistent loop over tiles)
//   block   -> workgroup of 256 lanes = 4 wavefronts in a 2 x 2 arrangement
//   thread  -> lane; its registers hold (BM/32)*(BN/32) MFMA accumulators
//   element -> 16x16 MFMA fragments (4 values per lane) and 16-byte loads
// A and B are double buffered in LDS: the global loads of k-tile t+1 are in
// flight while the matrix cores work on tile t, with one barrier per tile.
//
// LDS layouts (chosen for conflict-free 16-byte LDS traffic):
//   A: [BK/VEC][BM+2][VEC]  -- VEC = 16/sizeof(T) consecutive k values of one
//      row form one 16-byte chunk, written as loaded from row-major A and read
//      back with one ds_read_b128 that feeds VEC MFMAs.
//   B: [BK][BN+PB]          -- row-major like B in HBM.
// Transposed operands (op(A) = A^T with A stored k x m, op(B) = B^T with B
// stored n x k) swap layouts: a stored row of A^T is a k row of the tile, so
// it is staged like B ([BK][BM+PB], read one value per MFMA), and a stored
// row of B^T runs along k, so it is staged like A ([BK/VEC][BN+PA][VEC], read
// one 16-byte chunk per VEC MFMAs).
// Fragment k mapping: lane group g = lane/16 supplies k = VEC*(4r+g)+v to the
// v-th MFMA of round r on both operands, so A and B always agree on k, and
// every output sums its products in the same order for every layout.
#pragma once

#include "common.h"

namespace mg {

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4v acc_t;
  typedef d2v vec_t;  // one 16-byte chunk
  static constexpr int VEC = 2;
  static constexpr int BK = 16;
  static constexpr int PB = 8;  // B row pitch = BN + 8 doubles
  // Row (within the 16x16 block) of accumulator register r of lane group g.
  __device__ static __forceinline__ int row_of(int g, int r) { return 4 * r + g; }
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  typedef f4v acc_t;
  typedef f4v vec_t;
  static constexpr int VEC = 4;
  static constexpr int BK = 32;
  static constexpr int PB = 4;
  __device__ static __forceinline__ int row_of(int g, int r) { return 4 * g + r; }
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

template <typename T>
struct GemmArgs {
  const T *A;
  const T *B;
  T *C;
  int64_t lda, ldb, ldc;
  int m, n, k;
  T alpha, beta;
};

constexpr int kTileThreads = 256;

// Macro-tile BM x BN computed by WGM x WGN wavefronts (each a WM x WN wave
// tile of 16x16 MFMA blocks), k-step BK = BKM times the type's base step.
template <typename T, int BM, int BN, int WGM = 2, int WGN = 2, int BKM = 1, bool TA = false,
          bool TB = false>
struct TileShape {
  typedef Mfma<T> M;
  static constexpr int THREADS = 64 * WGM * WGN;
  static constexpr int VEC = M::VEC;
  static constexpr int BK = M::BK * BKM;
  static constexpr int ACH = BK / VEC;  // A chunks per tile row
  // A chunk-row pitch BM + PA: with ACH chunks per row written by consecutive
  // lanes, PA = 16 / ACH spreads the 16 lanes of a 16-byte LDS write over
  // all 64 banks.
  static constexpr int PA = 16 / ACH;
  static constexpr int PB = M::PB;
  static constexpr int WM = BM / WGM, WN = BN / WGN;  // wave tile
  static constexpr int FM = WM / 16, FN = WN / 16;    // MFMA blocks per wave
  static constexpr int A_CHUNKS = BM * BK / VEC;      // 16-byte chunks per A tile
  static constexpr int B_CHUNKS = BK * BN / VEC;
  static constexpr int NA = A_CHUNKS / THREADS;  // per thread
  static constexpr int NB = B_CHUNKS / THREADS;
  static constexpr int A_STAGE = TA ? BK * (BM + PB) : ACH * (BM + PA) * VEC;  // elements
  static constexpr int B_STAGE = TB ? ACH * (BN + PA) * VEC : BK * (BN + PB);
  static constexpr int STAGE = A_STAGE + B_STAGE;
  static constexpr size_t LDS_BYTES = 2 * STAGE * sizeof(T);
  static_assert(WM % 16 == 0 && WN % 16 == 0 && FM >= 1 && FN >= 1, "wave tile of 16x16 blocks");
  static_assert(ACH <= 16 && 16 % ACH == 0, "A chunks per row");
  static_assert(NA >= 1 && NB >= 1 && A_CHUNKS % THREADS == 0 && B_CHUNKS % THREADS == 0,
                "every thread loads whole chunks");
  static_assert(ACH % 4 == 0, "k rounds of 4 lane groups");
};

// Loads one 16-byte chunk of a row: `left` elements remain in the row from p.
template <typename T, bool VEC_OK>
__device__ __forceinline__ typename Mfma<T>::vec_t load_chunk(const T *p, bool ok, int left) {
  typedef typename Mfma<T>::vec_t V;
  constexpr int VEC = Mfma<T>::VEC;
  V r = {};
  if (VEC_OK && ok && left >= VEC) {
    r = *reinterpret_cast<const V *>(p);
  } else if (ok) {
#pragma unroll
    for (int v = 0; v < VEC; ++v)
      if (v < left) r[v] = p[v];
  }
  return r;
}

// Swap with the neighbouring lane (lane ^ 1) through DPP quad_perm [1,0,3,2].
__device__ __forceinline__ double dpp_swap1(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
  const int hi2 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

// Output row of accumulator register r of lane group gq in block row i.
// PA (paired block rows, FP64 direct-load tiles with a transposed A): block
// rows 2p and 2p+1 hold the even and odd rows of a 32-row span.
template <bool PA>
__device__ __forceinline__ int f64_out_row(int row0, int i, int gq, int r) {
  return PA ? row0 + 32 * (i >> 1) + 2 * Mfma<double>::row_of(gq, r) + (i & 1)
            : row0 + 16 * i + Mfma<double>::row_of(gq, r);
}

// C tile epilogue for a wave's FM x FN grid of 16x16 blocks whose top-left
// output is (row0, col0): out = alpha*acc + beta*C (C unread when beta == 0).
// In block (i, j), lane l holds column l%16 of rows row_of(l/16, r).  One
// block row i at a time, all its C loads are issued before its first store,
// so they are in flight together instead of each waiting behind the previous
// store (and the extra registers stay at one block row's worth).
// FP64: neighbouring lanes (same rows, columns c and c+1) swap one value each
// so that each lane owns a 16-byte pair of adjacent columns of one row.
template <typename T, bool VEC_OK>
struct Epilogue;

template <bool VEC_OK>
struct Epilogue<double, VEC_OK> {
  template <int FM, int FN, int AM, int AN, bool PA = false>
  __device__ static __forceinline__ void store(const GemmArgs<double> &g,
                                               const d4v (&acc)[AM][AN], int row0, int col0,
                                               int lane) {
    const int gq = lane >> 4, j = lane & 15;
    const bool odd = j & 1;
    const bool use_c = g.beta != 0.0;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      d2v v[FN][2], c[FN][2];
#pragma unroll
      for (int jb = 0; jb < FN; ++jb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = 2 * h;
          const double send = odd ? acc[i][jb][r] : acc[i][jb][r + 1];
          const double got = dpp_swap1(send);
          v[jb][h][0] = odd ? got : acc[i][jb][r];
          v[jb][h][1] = odd ? acc[i][jb][r + 1] : got;
        }
#pragma unroll
      for (int jb = 0; jb < FN; ++jb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = f64_out_row<PA>(row0, i, gq, 2 * h + (odd ? 1 : 0));
          const int col = col0 + 16 * jb + (j & ~1);
          c[jb][h] = d2v{0.0, 0.0};
          if (!use_c || row >= g.m) continue;
          const double *p = g.C + (int64_t)row * g.ldc + col;
          if (VEC_OK && col + 1 < g.n) {
            c[jb][h] = *reinterpret_cast<const d2v *>(p);
          } else {
            if (col < g.n) c[jb][h][0] = p[0];
            if (col + 1 < g.n) c[jb][h][1] = p[1];
          }
        }
#pragma unroll
      for (int jb = 0; jb < FN; ++jb)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int row = f64_out_row<PA>(row0, i, gq, 2 * h + (odd ? 1 : 0));
          const int col = col0 + 16 * jb + (j & ~1);
          if (row >= g.m) continue;
          d2v o;
#pragma unroll
          for (int e = 0; e < 2; ++e)
            o[e] = use_c ? fma(g.alpha, v[jb][h][e], g.beta * c[jb][h][e]) : g.alpha * v[jb][h][e];
          double *p = g.C + (int64_t)row * g.ldc + col;
          if (VEC_OK && col + 1 < g.n) {
            *reinterpret_cast<d2v *>(p) = o;
          } else {
            if (col < g.n) p[0] = o[0];
            if (col + 1 < g.n) p[1] = o[1];
          }
        }
    }
  }
};

// Epilogue of the column-paired FP64 fragment layout: block columns 2p and
// 2p+1 of a wave hold the even and odd columns of one 32-column span, so
// lane l owns columns 32p + 2(l%16) and 32p + 2(l%16) + 1 of each of its rows:
// one 16-byte C load and store per pair, no lane exchange.  C 16-byte aligned.
template <int FM, int FN, int AM, int AN, bool PA = false>
__device__ __forceinline__ void store_paired_f64(const GemmArgs<double> &g,
                                                 const d4v (&acc)[AM][AN], int row0, int col0,
                                                 int lane) {
  static_assert(FN % 2 == 0, "pairs of block columns");
  const int gq = lane >> 4, l16 = lane & 15;
  const bool use_c = g.beta != 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    d2v c[FN / 2][4];
#pragma unroll
    for (int p = 0; p < FN / 2; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = f64_out_row<PA>(row0, i, gq, r);
        const int col = col0 + 32 * p + 2 * l16;
        c[p][r] = d2v{0.0, 0.0};
        if (!use_c || row >= g.m) continue;
        const double *q = g.C + (int64_t)row * g.ldc + col;
        if (col + 1 < g.n) c[p][r] = *reinterpret_cast<const d2v *>(q);
        else if (col < g.n) c[p][r][0] = q[0];
      }
#pragma unroll
    for (int p = 0; p < FN / 2; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = f64_out_row<PA>(row0, i, gq, r);
        const int col = col0 + 32 * p + 2 * l16;
        if (row >= g.m) continue;
        d2v o;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const double v = acc[i][2 * p + e][r];
          o[e] = use_c ? fma(g.alpha, v, g.beta * c[p][r][e]) : g.alpha * v;
        }
        double *q = g.C + (int64_t)row * g.ldc + col;
        if (col + 1 < g.n) *reinterpret_cast<d2v *>(q) = o;
        else if (col < g.n) q[0] = o[0];
      }
  }
}

template <bool VEC_OK>
struct Epilogue<float, VEC_OK> {
  template <int FM, int FN, int AM, int AN>
  __device__ static __forceinline__ void store(const GemmArgs<float> &g,
                                               const f4v (&acc)[AM][AN], int row0, int col0,
                                               int lane) {
    const int gq = lane >> 4, j = lane & 15;
    const bool use_c = g.beta != 0.0f;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      float c[FN][4];
#pragma unroll
      for (int jb = 0; jb < FN; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + 16 * i + Mfma<float>::row_of(gq, r), col = col0 + 16 * jb + j;
          c[jb][r] = 0.0f;
          if (use_c && row < g.m && col < g.n) c[jb][r] = g.C[(int64_t)row * g.ldc + col];
        }
#pragma unroll
      for (int jb = 0; jb < FN; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + 16 * i + Mfma<float>::row_of(gq, r), col = col0 + 16 * jb + j;
          if (row < g.m && col < g.n)
            g.C[(int64_t)row * g.ldc + col] =
                use_c ? fmaf(g.alpha, acc[i][jb][r], g.beta * c[jb][r]) : g.alpha * acc[i][jb][r];
        }
    }
  }
};

// Computes the BM x BN tile of C whose top-left output is (m0, n0) of
// C <- alpha*op(A)*op(B) + beta*C (op = transpose when TA / TB is set).
// `smem` holds 2 stages of TileShape::STAGE elements.  All THREADS lanes of
// the workgroup must call this together (it contains barriers).
template <typename T, int BM, int BN, bool VEC_OK, int WGM = 2, int WGN = 2, int BKM = 1,
          bool TA = false, bool TB = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T> &g, int m0, int n0, T *smem) {
  typedef TileShape<T, BM, BN, WGM, WGN, BKM, TA, TB> S;
  typedef Mfma<T> M;
  typedef typename M::vec_t V;
  typedef typename M::acc_t Acc;
  constexpr int VEC = S::VEC, BK = S::BK;
  constexpr int ACH = S::ACH;    // k chunks per tile row of A (and of stored B^T)
  constexpr int BCH = BN / VEC;  // n chunks per k row of B
  constexpr int MCH = BM / VEC;  // m chunks per k row of stored A^T

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * S::WM, wn0 = (wave % WGN) * S::WN;
  const int gq = lane >> 4, l16 = lane & 15;

  // Per-thread global chunk coordinates (fixed across k-tiles).
  // A: (a_i, a_j) = (tile row, k chunk); transposed: (k row, first m column).
  const T *pa[S::NA];
  bool a_ok[S::NA];
  int a_i[S::NA], a_j[S::NA], a_left[S::NA];
#pragma unroll
  for (int u = 0; u < S::NA; ++u) {
    const int q = tid + S::THREADS * u;
    if constexpr (!TA) {
      a_i[u] = q / ACH;
      a_j[u] = q % ACH;
      const int grow = m0 + a_i[u];
      a_ok[u] = grow < g.m;
      pa[u] = g.A + (int64_t)(a_ok[u] ? grow : 0) * g.lda + a_j[u] * VEC;
    } else {
      a_i[u] = q / MCH;
      a_j[u] = (q % MCH) * VEC;
      const int gcol = m0 + a_j[u];
      a_ok[u] = gcol < g.m;
      a_left[u] = g.m - gcol;
      pa[u] = g.A + (int64_t)a_i[u] * g.lda + (a_ok[u] ? gcol : 0);
    }
  }
  // B: (b_i, b_j) = (k row, first n column); transposed: (tile column, k chunk).
  const T *pb[S::NB];
  bool b_ok[S::NB];
  int b_i[S::NB], b_j[S::NB], b_left[S::NB];
#pragma unroll
  for (int u = 0; u < S::NB; ++u) {
    const int q = tid + S::THREADS * u;
    if constexpr (!TB) {
      b_i[u] = q / BCH;
      b_j[u] = (q % BCH) * VEC;
      const int gcol = n0 + b_j[u];
      b_ok[u] = gcol < g.n;
      b_left[u] = g.n - gcol;
      pb[u] = g.B + (int64_t)b_i[u] * g.ldb + (b_ok[u] ? gcol : 0);
    } else {
      b_i[u] = q / ACH;
      b_j[u] = q % ACH;
      const int gcol = n0 + b_i[u];
      b_ok[u] = gcol < g.n;
      pb[u] = g.B + (int64_t)(b_ok[u] ? gcol : 0) * g.ldb + b_j[u] * VEC;
    }
  }

  V ra[S::NA], rb[S::NB];
  auto load_tiles = [&](int kt) {
    const int kbase = kt * BK;
#pragma unroll
    for (int u = 0; u < S::NA; ++u) {
      if constexpr (!TA) {
        const int kk = kbase + a_j[u] * VEC;
        ra[u] = load_chunk<T, VEC_OK>(pa[u] + kbase, a_ok[u], g.k - kk);
      } else {
        const int kr = kbase + a_i[u];
        ra[u] = load_chunk<T, VEC_OK>(pa[u] + (int64_t)kbase * g.lda, a_ok[u] && kr < g.k,
                                      a_left[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < S::NB; ++u) {
      if constexpr (!TB) {
        const int kr = kbase + b_i[u];
        rb[u] = load_chunk<T, VEC_OK>(pb[u] + (int64_t)kbase * g.ldb, b_ok[u] && kr < g.k,
                                      b_left[u]);
      } else {
        const int kk = kbase + b_j[u] * VEC;
        rb[u] = load_chunk<T, VEC_OK>(pb[u] + kbase, b_ok[u], g.k - kk);
      }
    }
  };
  auto store_tiles = [&](int stage) {
    T *As = smem + stage * S::STAGE;
    T *Bs = As + S::A_STAGE;
#pragma unroll
    for (int u = 0; u < S::NA; ++u) {
      if constexpr (!TA)
        *reinterpret_cast<V *>(As + (a_j[u] * (BM + S::PA) + a_i[u]) * VEC) = ra[u];
      else
        *reinterpret_cast<V *>(As + a_i[u] * (BM + S::PB) + a_j[u]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < S::NB; ++u) {
      if constexpr (!TB)
        *reinterpret_cast<V *>(Bs + b_i[u] * (BN + S::PB) + b_j[u]) = rb[u];
      else
        *reinterpret_cast<V *>(Bs + (b_j[u] * (BN + S::PA) + b_i[u]) * VEC) = rb[u];
    }
  };

  Acc acc[S::FM][S::FN];
#pragma unroll
  for (int i = 0; i < S::FM; ++i)
#pragma unroll
    for (int j = 0; j < S::FN; ++j) acc[i][j] = Acc{};

  const int KT = (g.k + BK - 1) / BK;
  MG_LDS_POISON_STAGE(smem, 2 * S::STAGE * (int)sizeof(T));
  if (KT > 0) {
    load_tiles(0);
    store_tiles(0);
  }
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    // the other buffer is refilled after this step's products
    MG_LDS_POISON_STAGE(smem + (cur ^ 1) * S::STAGE, S::STAGE * (int)sizeof(T));
    if (kt + 1 < KT) load_tiles(kt + 1);
    const T *As = smem + cur * S::STAGE;
    const T *Bs = As + S::A_STAGE;
#pragma unroll
    for (int r = 0; r < ACH / 4; ++r) {
      const int kc = 4 * r + gq;  // this lane group's chunk
      V a[S::FM];
#pragma unroll
      for (int i = 0; i < S::FM; ++i) {
        if constexpr (!TA) {
          a[i] = *reinterpret_cast<const V *>(As + (kc * (BM + S::PA) + wm0 + 16 * i + l16) * VEC);
        } else {
#pragma unroll
          for (int v = 0; v < VEC; ++v)
            a[i][v] = As[(kc * VEC + v) * (BM + S::PB) + wm0 + 16 * i + l16];
        }
      }
      V bv[S::FN];  // transposed B: one chunk of VEC k values per block column
      if constexpr (TB) {
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
          bv[j] = *reinterpret_cast<const V *>(Bs + (kc * (BN + S::PA) + wn0 + 16 * j + l16) * VEC);
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        T b[S::FN];
#pragma unroll
        for (int j = 0; j < S::FN; ++j) {
          if constexpr (!TB)
            b[j] = Bs[(kc * VEC + v) * (BN + S::PB) + wn0 + 16 * j + l16];
          else
            b[j] = bv[j][v];
        }
#pragma unroll
        for (int i = 0; i < S::FM; ++i)
#pragma unroll
          for (int j = 0; j < S::FN; ++j) acc[i][j] = M::mma(a[i][v], b[j], acc[i][j]);
      }
    }
    if (kt + 1 < KT) store_tiles(cur ^ 1);
    __syncthreads();
  }

  Epilogue<T, VEC_OK>::template store<S::FM, S::FN>(g, acc, m0 + wm0, n0 + wn0, lane);
}

}  // namespace mg
