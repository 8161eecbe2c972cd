// Native GEMM tile fed by direct global->LDS loads (gfx950
// global_load_lds_dwordx4) into an NS-stage LDS ring.
//
// Same hierarchy as gemm_tile (Section 4.2.2 tiling: block = macro-tile of
// C, threads stage A/B tiles in shared memory, each lane accumulates MFMA
// fragments), but the loads of k-steps t+1 .. t+NS-1 are in flight while the
// matrix cores work on step t, and no registers or LDS write instructions are
// spent on staging: each lane's 16 bytes land at the wave's LDS base + 16*lane.
// Requires 16-byte aligned operands (base aligned, pitch a multiple of the
// 16-byte element count); ragged edges are read from clamped in-bounds
// chunks and never stored, and k past the problem's k is zeroed in LDS on
// both operands before the last step's multiply (the same sums as the
// zero-filled tail of the register-staged tile).
//
// One k-step covers 128 bytes of k (16 FP64 / 32 FP32 values).  LDS stage:
//   A [BM rows][128 B], 16-byte chunk c of row r stored at chunk c ^ ((r>>1)&7)
//     so the fragment reads of 16 consecutive rows hit distinct banks;
//   B [128/size rows of k][BN*size B], row-major like B in HBM, chunks XOR-
//     swizzled per k row so the four lane groups' rows of one fragment read
//     fall on different banks.
// Transposed operands keep the stored rows intact: A^T (stored k x m) lands
// as [k rows][BM*size B] with B's swizzle and is read one value per MFMA like
// B; B^T (stored n x k) lands as [BN rows][128 B] with A's swizzle and is read
// one 16-byte chunk per VEC MFMAs like A.  Stage sizes are the same.
#pragma once

#include "gemm_tile.h"

namespace mg {

// KS = 2 runs two groups of WGM x WGN wavefronts on the same outputs, each
// taking half of every k-step's values (16-byte k chunks 0-3 and 4-7); the
// second group's sums are added to the first's through LDS at the end.
template <typename T, int BM, int BN, int WGM, int WGN, int NS, int KS = 1>
struct DmaShape {
  static constexpr int SWAVES = WGM * WGN;     // wavefronts per k group
  static constexpr int WAVES = SWAVES * KS;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int ESZ = sizeof(T);
  static constexpr int VEC = 16 / ESZ;
  static constexpr int BK = 128 / ESZ;
  static constexpr int RB = BN * ESZ;          // B row bytes in LDS
  static constexpr int CPB = RB / 16;          // 16-byte chunks per B row
  static constexpr int RA = BM * ESZ;          // row bytes of a transposed A stage
  static constexpr int CPA = RA / 16;
  static constexpr int A_BYTES = BM * 128;
  static constexpr int STAGE = A_BYTES + 128 * BN;  // B block: BK rows of RB bytes
  static constexpr size_t RING_BYTES = (size_t)NS * STAGE;
  static constexpr size_t RED_BYTES = KS > 1 ? (size_t)BM * BN * ESZ : 0;  // k-group sums
  static constexpr size_t LDS_BYTES = RING_BYTES > RED_BYTES ? RING_BYTES : RED_BYTES;
  static constexpr int IA = BM / 8 / WAVES;    // 1 KB DMA instructions per wave, A
  static constexpr int IB = BN / 8 / WAVES;    // and B
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(IA >= 1 && IA * 8 * WAVES == BM, "whole A instructions per wave");
  static_assert(IB >= 1 && IB * 8 * WAVES == BN, "whole B instructions per wave");
  static_assert(FM >= 1 && FN >= 1 && WM % 16 == 0 && WN % 16 == 0, "16x16 blocks per wave");
  static_assert(CPB >= 8 && (CPB & (CPB - 1)) == 0, "B rows of 2^j >= 8 chunks");
  static_assert(NS >= 2 && LDS_BYTES <= 160 * 1024, "ring fits in LDS");
  static_assert(KS == 1 || KS == 2, "one or two k groups");
  // Wavefronts per SIMD the register allocation must leave room for (the
  // second __launch_bounds__ value): as many workgroups as the LDS ring
  // allows per CU, counted up to 2 per SIMD so large register tiles (a
  // 4-wave 128x128 tile holds 128 FP64 accumulators per lane) still get 256.
  static constexpr int WGS_PER_CU = (int)((160 * 1024) / LDS_BYTES);
  static constexpr int MINW = WGS_PER_CU * WAVES / 4 >= 2 ? 2 : 1;
};

__device__ __forceinline__ int dma_swz_a(int row, int c) { return c ^ ((row >> 1) & 7); }

// FP64 fragments read 8-byte values of 16 consecutive columns (128 B) from the
// rows 2(4r+g)+v of the four lane groups g: flip the 128-byte half by a bit
// that differs between any two of them.  FP32 reads 64 B from rows 4(4r+g)+v:
// rotate by 64-byte quarters with (row/4) mod 4.
template <typename T, int CPB>
__device__ __forceinline__ int dma_swz_b(int row, int c) {
  if (sizeof(T) == 8) return c ^ ((((row >> 1) ^ (row >> 2)) & 1) << 3);
  return c ^ ((((row >> 2) & 3) << 2) & (CPB - 1));
}

__device__ __forceinline__ void dma_lds16(const void *src, unsigned char *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0,
                                   0);
}

template <int N>
__device__ __forceinline__ void dma_wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 s_waitcnt encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[15:14]
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Waits until at most q k-steps' DMAs (DPS instructions each) are pending.
template <int DPS, int NS>
__device__ __forceinline__ void dma_wait_steps(int q) {
  if (q <= 0) dma_wait_vmcnt<0>();
  else if (q == 1 || NS <= 2) dma_wait_vmcnt<DPS>();
  else if (q == 2 || NS <= 3) dma_wait_vmcnt<2 * DPS>();
  else dma_wait_vmcnt<3 * DPS>();
}

template <typename T, int BM, int BN, int WGM, int WGN, int NS, bool TA = false, bool TB = false,
          int KS = 1>
__device__ __forceinline__ void gemm_dma_tile(const GemmArgs<T> &g, int m0, int n0,
                                              unsigned char *lds) {
  typedef DmaShape<T, BM, BN, WGM, WGN, NS, KS> S;
  typedef Mfma<T> M;
  typedef typename M::vec_t V;
  typedef typename M::acc_t Acc;
  constexpr int ESZ = S::ESZ, VEC = S::VEC, BK = S::BK;
  constexpr int DPS = S::IA + S::IB;  // DMA instructions per k-step per wave
  // FP64 with B in k rows: pair block columns 2p, 2p+1 on the even / odd
  // columns of a 32-column span, so one 16-byte LDS read feeds both.
  constexpr bool PAIR = ESZ == 8 && !TB && S::FN % 2 == 0;
  // FP64 with A in k rows (transposed A): pair block rows 2p, 2p+1 on the
  // even / odd rows of a 32-row span the same way.
  constexpr bool PAIRA = ESZ == 8 && TA && S::FM % 2 == 0;
  static_assert(!TA || (S::CPA >= 8 && (S::CPA & (S::CPA - 1)) == 0),
                "transposed A rows of 2^j >= 8 chunks");
  static_assert(ESZ == 4 || (S::CPB >= 16 && (!TA || S::CPA >= 16)), "FP64 swizzle flips bit 3");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sw = wave % S::SWAVES, kg = wave / S::SWAVES;  // output block, k group
  const int wm0 = (sw / WGN) * S::WM, wn0 = (sw % WGN) * S::WN;
  const int gq = lane >> 4, l16 = lane & 15;

  // Source of this lane's chunk in every DMA slot, without the k-step offset.
  // Rows of 128 B of k (A, or stored B^T): slot u covers rows 8q .. 8q+7
  // (q = wave*I + u), lane -> row 8q + lane/8, physical chunk lane%8 holding
  // logical chunk c; koff = c*VEC.  Rows of k (B, or stored A^T): slot u
  // covers stage bytes [1024q, 1024q + 1024); koff = the k row.  Rows past
  // the matrix and chunks past its columns are clamped to the last valid ones.
  const char *A = reinterpret_cast<const char *>(g.A);
  const char *B = reinterpret_cast<const char *>(g.B);
  const char *asrc[S::IA];
  int akofs[S::IA];
#pragma unroll
  for (int u = 0; u < S::IA; ++u) {
    if constexpr (!TA) {
      const int row = 8 * (wave * S::IA + u) + (lane >> 3);
      akofs[u] = dma_swz_a(row, lane & 7) * VEC;
      const int gr = min(m0 + row, g.m - 1);
      asrc[u] = A + ((int64_t)gr * g.lda + akofs[u]) * ESZ;
    } else {
      const int o = (wave * S::IA + u) * 1024 + lane * 16;
      const int row = o / S::RA;
      const int c = dma_swz_b<T, S::CPA>(row, (o % S::RA) >> 4);
      akofs[u] = row;
      const int gc = min(m0 + c * VEC, ((g.m - 1) / VEC) * VEC);
      asrc[u] = A + ((int64_t)row * g.lda + gc) * ESZ;
    }
  }
  const char *bsrc[S::IB];
  int bkrow[S::IB];
#pragma unroll
  for (int u = 0; u < S::IB; ++u) {
    if constexpr (!TB) {
      const int o = (wave * S::IB + u) * 1024 + lane * 16;
      const int row = o / S::RB;
      const int c = dma_swz_b<T, S::CPB>(row, (o % S::RB) >> 4);
      bkrow[u] = row;
      const int gc = min(n0 + c * VEC, ((g.n - 1) / VEC) * VEC);
      bsrc[u] = B + ((int64_t)row * g.ldb + gc) * ESZ;
    } else {
      const int row = 8 * (wave * S::IB + u) + (lane >> 3);
      bkrow[u] = dma_swz_a(row, lane & 7) * VEC;
      const int gr = min(n0 + row, g.n - 1);
      bsrc[u] = B + ((int64_t)gr * g.ldb + bkrow[u]) * ESZ;
    }
  }

  const int KT = (g.k + BK - 1) / BK;
  const int last_k_chunk = ((g.k - 1) / VEC) * VEC;
  // k-step offset of a slot: along the row (k-contiguous rows) or down the
  // rows (k rows); on the partial last step the k chunk / k row is clamped.
  auto src_k = [&](const char *src, int koff, int64_t ld, bool krows, int kbase,
                   bool tail) -> const char * {
    if (!krows) {
      if (!tail) return src + (int64_t)kbase * ESZ;
      const int kk = min(kbase + koff, last_k_chunk);
      return src + (int64_t)(kk - koff) * ESZ;
    }
    if (!tail) return src + (int64_t)kbase * ld * ESZ;
    const int kr = min(kbase + koff, g.k - 1);
    return src + (int64_t)(kr - koff) * ld * ESZ;
  };
  auto issue = [&](int kt) {
    const int kbase = kt * BK;
    unsigned char *la = lds + (kt % NS) * S::STAGE;
    unsigned char *lb = la + S::A_BYTES;
    if (kbase + BK <= g.k) {
#pragma unroll
      for (int u = 0; u < S::IA; ++u)
        dma_lds16(src_k(asrc[u], akofs[u], g.lda, TA, kbase, false),
                  la + (wave * S::IA + u) * 1024);
#pragma unroll
      for (int u = 0; u < S::IB; ++u)
        dma_lds16(src_k(bsrc[u], bkrow[u], g.ldb, !TB, kbase, false),
                  lb + (wave * S::IB + u) * 1024);
    } else {
#pragma unroll
      for (int u = 0; u < S::IA; ++u)
        dma_lds16(src_k(asrc[u], akofs[u], g.lda, TA, kbase, true),
                  la + (wave * S::IA + u) * 1024);
#pragma unroll
      for (int u = 0; u < S::IB; ++u)
        dma_lds16(src_k(bsrc[u], bkrow[u], g.ldb, !TB, kbase, true),
                  lb + (wave * S::IB + u) * 1024);
    }
  };

  Acc acc[S::FM][S::FN];
#pragma unroll
  for (int i = 0; i < S::FM; ++i)
#pragma unroll
    for (int j = 0; j < S::FN; ++j) acc[i][j] = Acc{};

  auto compute = [&](const unsigned char *As, const unsigned char *Bs) {
#pragma unroll
    for (int rr = 0; rr < 2 / KS; ++rr) {
      const int r = KS == 2 ? kg : rr;  // with two k groups, this group's half of the step
      const int kc = 4 * r + gq;        // this lane group's 16-byte k chunk
      V a[S::FM];
#pragma unroll
      for (int i = 0; i < S::FM; ++i) {
        const int row = wm0 + 16 * i + l16;
        if constexpr (!TA) {
          a[i] = *reinterpret_cast<const V *>(As + row * 128 + dma_swz_a(row, kc) * 16);
        } else if constexpr (PAIRA) {
          if (i % 2 == 0) {  // rows wm0 + 32p + 2*l16 (block 2p) and +1 (block 2p+1)
            const int chunk = ((wm0 + 16 * i) >> 1) + l16;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
              const int kr = kc * VEC + v;
              const V aa = *reinterpret_cast<const V *>(As + kr * S::RA +
                                                        dma_swz_b<T, S::CPA>(kr, chunk) * 16);
              a[i][v] = aa[0];
              a[i + 1][v] = aa[1];
            }
          }
        } else {
          const int byte = row * ESZ;
#pragma unroll
          for (int v = 0; v < VEC; ++v) {
            const int kr = kc * VEC + v;
            a[i][v] = *reinterpret_cast<const T *>(
                As + kr * S::RA + dma_swz_b<T, S::CPA>(kr, byte >> 4) * 16 + (byte & 15));
          }
        }
      }
      if constexpr (PAIR) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const int kr = kc * VEC + v;
          T b[S::FN];
#pragma unroll
          for (int p = 0; p < S::FN / 2; ++p) {
            const int chunk = ((wn0 + 32 * p) >> 1) + l16;  // columns wn0 + 32p + 2*l16, +1
            const V bb = *reinterpret_cast<const V *>(Bs + kr * S::RB +
                                                      dma_swz_b<T, S::CPB>(kr, chunk) * 16);
            b[2 * p] = bb[0];
            b[2 * p + 1] = bb[1];
          }
#pragma unroll
          for (int i = 0; i < S::FM; ++i)
#pragma unroll
            for (int j = 0; j < S::FN; ++j) acc[i][j] = M::mma(a[i][v], b[j], acc[i][j]);
        }
        continue;
      }
      V bv[S::FN];  // transposed B: one chunk of VEC k values per block column
      if constexpr (TB) {
#pragma unroll
        for (int j = 0; j < S::FN; ++j) {
          const int col = wn0 + 16 * j + l16;
          bv[j] = *reinterpret_cast<const V *>(Bs + col * 128 + dma_swz_a(col, kc) * 16);
        }
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int kr = kc * VEC + v;
        T b[S::FN];
#pragma unroll
        for (int j = 0; j < S::FN; ++j) {
          if constexpr (!TB) {
            const int byte = (wn0 + 16 * j + l16) * ESZ;
            b[j] = *reinterpret_cast<const T *>(Bs + kr * S::RB +
                                                dma_swz_b<T, S::CPB>(kr, byte >> 4) * 16 +
                                                (byte & 15));
          } else {
            b[j] = bv[j][v];
          }
        }
#pragma unroll
        for (int i = 0; i < S::FM; ++i)
#pragma unroll
          for (int j = 0; j < S::FN; ++j) acc[i][j] = M::mma(a[i][v], b[j], acc[i][j]);
      }
    }
  };

  // Last, partial k-step: zero every k >= kvalid of the landed stage (A
  // columns, B rows), so values read from clamped addresses never reach the
  // sums; the same zeros the register-staged tile loads past k.
  auto zero_krows = [&](unsigned char *X, int cp, int kvalid) {  // [k rows][cp chunks]
    for (int e = tid; e < BK * cp; e += S::THREADS)
      if (e / cp >= kvalid) *reinterpret_cast<V *>(X + e * 16) = V{};
  };
  auto zero_kcols = [&](unsigned char *X, int rows, int kvalid) {  // [rows][128 B of k]
    for (int e = tid; e < rows * 8; e += S::THREADS) {
      const int row = e >> 3, c = e & 7;
      if ((c + 1) * VEC <= kvalid) continue;
      T *p = reinterpret_cast<T *>(X + row * 128 + dma_swz_a(row, c) * 16);
#pragma unroll
      for (int v = 0; v < VEC; ++v)
        if (c * VEC + v >= kvalid) p[v] = T(0);
    }
  };
  auto zero_tail = [&](unsigned char *As, unsigned char *Bs, int kvalid) {
    if constexpr (!TA) zero_kcols(As, BM, kvalid);
    else zero_krows(As, S::CPA, kvalid);
    if constexpr (!TB) zero_krows(Bs, S::CPB, kvalid);
    else zero_kcols(Bs, BN, kvalid);
  };

  MG_LDS_POISON_STAGE(lds, NS * S::STAGE);
#pragma unroll
  for (int q = 0; q < NS - 1; ++q)
    if (q < KT) issue(q);
  for (int kt = 0; kt < KT; ++kt) {
    // step kt has landed once only the later issued steps may be pending
    dma_wait_steps<DPS, NS>(min(KT - 1, kt + NS - 2) - kt);
    __builtin_amdgcn_s_barrier();
    if (kt + NS - 1 < KT) {
      MG_LDS_POISON_STAGE(lds + ((kt + NS - 1) % NS) * S::STAGE, S::STAGE);
      issue(kt + NS - 1);
    }
    unsigned char *As = lds + (kt % NS) * S::STAGE;
    unsigned char *Bs = As + S::A_BYTES;
    const int kvalid = g.k - kt * BK;
    if (kvalid < BK) {  // only the last step; nothing is in flight any more
      zero_tail(As, Bs, kvalid);
      __syncthreads();
    }
    compute(As, Bs);
  }

  if constexpr (KS == 2) {
    // k group 1 hands its sums to group 0 through LDS (the ring is free once
    // every wave is past its last step); group 0 adds them and stores.
    constexpr int NA = sizeof(Acc) / sizeof(T);
    T *red = reinterpret_cast<T *>(lds) + (size_t)sw * S::FM * S::FN * NA * 64 + lane;
    __syncthreads();
    if (kg == 1) {
#pragma unroll
      for (int i = 0; i < S::FM; ++i)
#pragma unroll
        for (int j = 0; j < S::FN; ++j)
#pragma unroll
          for (int e = 0; e < NA; ++e) red[((i * S::FN + j) * NA + e) * 64] = acc[i][j][e];
    }
    __syncthreads();
    if (kg == 1) return;
#pragma unroll
    for (int i = 0; i < S::FM; ++i)
#pragma unroll
      for (int j = 0; j < S::FN; ++j)
#pragma unroll
        for (int e = 0; e < NA; ++e) acc[i][j][e] += red[((i * S::FN + j) * NA + e) * 64];
  }

  if constexpr (PAIR)
    store_paired_f64<S::FM, S::FN, S::FM, S::FN, PAIRA>(g, acc, m0 + wm0, n0 + wn0, lane);
  else if constexpr (ESZ == 8)
    Epilogue<T, true>::template store<S::FM, S::FN, S::FM, S::FN, PAIRA>(g, acc, m0 + wm0,
                                                                          n0 + wn0, lane);
  else
    Epilogue<T, true>::template store<S::FM, S::FN>(g, acc, m0 + wm0, n0 + wn0, lane);
}

}  // namespace mg
