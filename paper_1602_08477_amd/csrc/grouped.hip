// Batched uneven GEMMs in one persistent launch.
//
// A plan turns a list of independent problems C_i <- alpha_i A_i B_i +
// beta_i C_i into a device work list of macro-tiles (each record carries its
// problem's arguments, tile coordinates and a tile class from the tuning
// table), sorted longest first.  One persistent kernel of (CUs x occupancy)
// workgroups deals the list out in rounds of G tiles, alternating direction
// (workgroup b takes tile b of round 0, G-1-b of round 1, ...: with the list
// in decreasing cost every workgroup ends up with about the same work) and
// runs the same per-tile arithmetic as the single-problem kernel,
// so a problem's result does not depend on what else is in the batch.  Each
// workgroup streams its tiles' k-steps through an LDS ring that is filled two
// steps ahead, across tile boundaries.  The launch is captured once in a HIP
// graph and replayed.
//
// In the paper's terms (Section 3.2): blocks are independent and are never
// synchronised with each other; they share nothing but the read-only list.
#include "grouped.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <type_traits>
#include <vector>

#include "gemm_tile.h"

namespace mg {

namespace {

// Tile classes of the persistent kernel (work divisions per problem).
constexpr int kClsBM[kNumGroupedClasses] = {64, 64, 32};
constexpr int kClsBN[kNumGroupedClasses] = {64, 32, 32};
constexpr int kScaleCls = 15;  // C <- beta*C only (alpha == 0 or k == 0)
constexpr int kScaleTile = 64;

// One macro-tile of work: the problem's arguments inline (one load per tile).
template <typename T>
struct GTileRec {
  GemmArgs<T> g;
  int tm, tn;
  int cls;  // class | (16-byte aligned rows: C << 4, A << 5, B << 6)
  int pad;
};

template <typename T>
__device__ __forceinline__ void scale_tile(const GemmArgs<T> &g, int m0, int n0) {
  for (int e = threadIdx.x; e < kScaleTile * kScaleTile; e += kTileThreads) {
    const int i = m0 + e / kScaleTile, j = n0 + e % kScaleTile;
    if (i < g.m && j < g.n) {
      T *p = g.C + (int64_t)i * g.ldc + j;
      *p = g.beta == T(0) ? T(0) : g.beta * *p;
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent kernel with a ring of direct global->LDS loads.
//
// Each workgroup walks its dealt tiles as one stream of k-steps.  A
// load cursor runs NS-1 steps ahead of the compute cursor and fills an
// NS-stage LDS ring with global_load_lds (4 bytes per lane, so any leading
// dimension and any element alignment is accepted), across tile boundaries:
// the first k-steps of the next tile arrive while the current tile finishes.
// No staging registers are used, which leaves room for two workgroups per CU.
//
// Edges: rows past m and columns past n are read from clamped in-bounds
// addresses and never stored; k past the problem's k is read from a clamped
// address and zeroed on both operands before the multiply.
//
// LDS stage: A block [BM rows][128 B] (BK = 128 B of k per step), its 16-byte
// chunks XOR-swizzled per row so that the fragment reads of 16 rows hit
// distinct banks; B block [BK/VEC][BN][VEC]: the VEC consecutive k of one
// column form one 16-byte chunk, so a lane reads the B values of VEC MFMAs
// with one 16-byte load and 16 lanes read 256 contiguous bytes.
constexpr int kGdStageA = 64 * 128;
constexpr int kGdStageB = 8192;
constexpr int kGdStage = kGdStageA + kGdStageB;
constexpr int kGdNS = 3;
constexpr int kGdMinBlocks = 3;  // workgroups per CU the register budget is sized for
// A step issues at most 16 DMA instructions; the waits below cover the
// steps in flight behind the one being consumed.
static_assert((kGdNS - 2) * 16 <= 48, "ring deeper than the vmcnt waits cover");

__device__ __forceinline__ int gd_bm(int cls) { return cls == 2 ? 32 : 64; }
__device__ __forceinline__ int gd_bn(int cls) { return cls == 0 ? 64 : 32; }

// Physical 16-byte chunk of logical chunk c in A row `row`.
__device__ __forceinline__ int gd_swz_a(int row, int c) { return c ^ ((row >> 1) & 7); }

template <int N>
__device__ __forceinline__ void gd_wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ void gd_dma4(const void *src, unsigned char *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 4, 0,
                                   0);
}

// This lane's source addresses of one tile for every DMA slot, without the
// k offset of the step: slot u of A covers tile row 2q + lane/32 (q = wave*ia
// + u), slot u of B covers LDS bytes [256q, 256q + 256) of the B block.
// Rows past m and columns past n are clamped to the last valid one.
template <typename T>
struct GdSlots {
  const char *a[8];
  const char *b[8];
  int ia, ib;
};

// Logical k offset (elements) of 16-byte A slot u, and k row of 16-byte B
// slot u (a 16-byte B slot covers 1 KB of the row-major block).
template <typename T>
__device__ __forceinline__ int gd_a16_kofs(int wave, int ia, int u, int lane) {
  const int row = 8 * (wave * ia + u) + (lane >> 3);
  return gd_swz_a(row, lane & 7) * (16 / (int)sizeof(T));
}
template <typename T>
__device__ __forceinline__ int gd_b16_krow(int wave, int ib, int u, int lane, int bn) {
  return ((wave * ib + u) * 1024 + lane * 16) / (bn * (int)sizeof(T));
}

// Row-major B block of a 16-byte-B tile: [BK rows][BN*size B], chunk c of
// row r stored at gd_swz_b(r, c), which puts the rows read together by the
// four lane groups of a fragment read (2 apart for FP64, 4 for FP32) on
// different halves of the banks.
template <typename T>
__device__ __forceinline__ int gd_swz_b(int row, int c, int cpb) {  // cpb: chunks per row, >= 8
  if (sizeof(T) == 8) return c ^ ((((row >> 1) ^ (row >> 2)) & 1) << 3);
  return c ^ ((((row >> 2) & 3) << 2) & (cpb - 1));
}

__device__ __forceinline__ void gd_dma16(const void *src, unsigned char *lds_dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)lds_dst, 16, 0,
                                   0);
}

template <typename T>
__device__ __forceinline__ int gd_a_kofs(int wave, int ia, int u, int lane) {
  constexpr int ESZ = sizeof(T), VEC = 16 / ESZ;
  const int row = 2 * (wave * ia + u) + (lane >> 5);
  return gd_swz_a(row, (lane & 31) >> 2) * VEC + ((lane & 3) * 4) / ESZ;
}

// B block byte o = ((kc*bn + col)*VEC + e)*size + (4-byte half): slot u of a
// wave covers o in [256q, 256q + 256), q = wave*ib + u, lane at 4*lane.
template <typename T>
__device__ __forceinline__ int gd_b_krow(int wave, int ib, int u, int lane, int bn) {
  constexpr int ESZ = sizeof(T), VEC = 16 / ESZ;
  const int o = (wave * ib + u) * 256 + lane * 4;
  return ((o >> 4) >> (bn == 64 ? 6 : 5)) * VEC + (o & 15) / ESZ;  // kc*VEC + e
}

template <typename T>
__device__ __forceinline__ int gd_b_col(int wave, int ib, int u, int lane, int bn) {
  const int o = (wave * ib + u) * 256 + lane * 4;
  return (o >> 4) & (bn - 1);
}

// A16: A's rows are 16-byte aligned (pitch a multiple of 16 bytes, aligned
// base): its slots become 16-byte loads, lane -> row 8q + lane/8, physical
// chunk lane%8 holding logical chunk gd_swz_a(row, lane%8) -- the same LDS
// contents as the 4-byte slots, in a quarter of the instructions.
// 16-byte slots are built for FP64 only (kGd16 false: the FP32 kernel keeps
// the 4-byte loads alone, which measured faster for it).
template <typename T>
constexpr bool kGd16 = sizeof(T) == 8;

template <typename T>
__device__ __forceinline__ void gd_setup(GdSlots<T> &sl, const GemmArgs<T> &g, int cls, int m0,
                                         int n0, int wave, int lane, bool a16, bool b16) {
  constexpr int ESZ = sizeof(T), VEC = 16 / ESZ;
  a16 = kGd16<T> && a16;
  b16 = kGd16<T> && b16;
  const int bm = gd_bm(cls), bn = gd_bn(cls);
  sl.ib = b16 ? bn / 32 : bn / 8;
  const int boff = ((lane & 3) * 4) % ESZ;  // 4-byte half of an FP64 element
  const char *A = reinterpret_cast<const char *>(g.A);
  const char *B = reinterpret_cast<const char *>(g.B);
  // Every slot is written on both paths (the unused 16-byte ones hold the
  // 4-byte pointer): stores at fixed offsets keep the slot arrays in
  // registers instead of private memory.
  sl.ia = a16 ? bm / 32 : bm / 8;  // 16-byte: 8 rows per instruction, 4 waves
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int row4 = 2 * (wave * (bm / 8) + u) + (lane >> 5);
    const char *p = A + ((int64_t)min(m0 + row4, g.m - 1) * g.lda +
                         gd_a_kofs<T>(wave, bm / 8, u, lane)) * ESZ + boff;
    if (kGd16<T> && u < 2) {
      const int row16 = 8 * (wave * (bm / 32) + u) + (lane >> 3);
      const char *q = A + ((int64_t)min(m0 + row16, g.m - 1) * g.lda +
                           gd_a16_kofs<T>(wave, bm / 32, u, lane)) * ESZ;
      p = a16 ? q : p;
    }
    sl.a[u] = p;
  }
  const int rb = bn * ESZ, last_col = ((g.n - 1) / VEC) * VEC;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int ib4 = bn / 8;
    const int col = gd_b_col<T>(wave, ib4, u, lane, bn);
    const char *p = B + ((int64_t)gd_b_krow<T>(wave, ib4, u, lane, bn) * g.ldb +
                         min(n0 + col, g.n - 1)) * ESZ + boff;
    if (kGd16<T> && u < 2) {  // 16-byte: 1 KB (one or two k rows of the block) per instruction
      const int o = (wave * (bn / 32) + u) * 1024 + lane * 16;
      const int row = o / rb;
      const int c = gd_swz_b<T>(row, (o % rb) >> 4, rb >> 4);
      const char *q = B + ((int64_t)row * g.ldb + min(n0 + c * VEC, last_col)) * ESZ;
      p = b16 ? q : p;
    }
    sl.b[u] = p;
  }
}

// Issues this wave's share of the k-step at `kbase` (A and B blocks) into
// `stage`; returns the number of DMA instructions issued.
// Whole steps add one uniform offset per slot; the last, partial step of a
// tile clamps k to the problem's last column of A / row of B.
template <typename T>
__device__ __forceinline__ int gd_issue(const GdSlots<T> &sl, const GemmArgs<T> &g, int cls_bits,
                                        int kbase, unsigned char *stage, int wave, int lane) {
  constexpr int ESZ = sizeof(T), BK = 128 / ESZ;
  const int cls = cls_bits & 15;
  const bool a16 = kGd16<T> && ((cls_bits >> 5) & 1), b16 = kGd16<T> && ((cls_bits >> 6) & 1);
  const bool whole = kbase + BK <= g.k;
  const int64_t bstep = (int64_t)kbase * g.ldb * ESZ;
  if (a16) {
    const int last_chunk = ((g.k - 1) / (16 / ESZ)) * (16 / ESZ);
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (u < sl.ia) {
        const char *src = sl.a[u] + (int64_t)kbase * ESZ;
        if (!whole) {
          const int ko = gd_a16_kofs<T>(wave, sl.ia, u, lane);
          src = sl.a[u] + (int64_t)(min(kbase + ko, last_chunk) - ko) * ESZ;
        }
        gd_dma16(src, stage + (wave * sl.ia + u) * 1024);
      }
  }
  if (b16) {
    const int bn = gd_bn(cls);
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (u < sl.ib) {
        const char *src = sl.b[u] + bstep;
        if (!whole) {
          const int kr = gd_b16_krow<T>(wave, sl.ib, u, lane, bn);
          src = sl.b[u] + (int64_t)(min(kbase + kr, g.k - 1) - kr) * g.ldb * ESZ;
        }
        gd_dma16(src, stage + kGdStageA + (wave * sl.ib + u) * 1024);
      }
  }
  if (whole) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!a16 && u < sl.ia)
        gd_dma4(sl.a[u] + (int64_t)kbase * ESZ, stage + (wave * sl.ia + u) * 256);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!b16 && u < sl.ib)
        gd_dma4(sl.b[u] + bstep, stage + kGdStageA + (wave * sl.ib + u) * 256);
  } else {
    const int klast = g.k - 1;
    const int bn = gd_bn(cls);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!a16 && u < sl.ia) {
        const int ko = gd_a_kofs<T>(wave, sl.ia, u, lane);
        gd_dma4(sl.a[u] + (int64_t)(min(kbase + ko, klast) - ko) * ESZ,
                stage + (wave * sl.ia + u) * 256);
      }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!b16 && u < sl.ib) {
        const int kr = gd_b_krow<T>(wave, sl.ib, u, lane, bn);
        gd_dma4(sl.b[u] + (int64_t)(min(kbase + kr, klast) - kr) * g.ldb * ESZ,
                stage + kGdStageA + (wave * sl.ib + u) * 256);
      }
  }
  return sl.ia + sl.ib;
}

// One k-step of a BM x BN tile from an LDS stage.  TAIL: only the first
// `kvalid` k of the step belong to the problem; the rest is zeroed on both
// operands (values read from clamped addresses never reach the sums).
// BROW: the step's B block is row-major (a 16-byte-B tile): one value per
// MFMA is read instead of one 16-byte chunk of VEC k values per column.
template <typename T, int BM, int BN, bool TAIL, bool BROW>
__device__ __forceinline__ void gd_compute(typename Mfma<T>::acc_t (&acc)[BM / 32][BN / 32],
                                           const unsigned char *As, const unsigned char *Bs,
                                           int wave, int lane, int kvalid) {
  typedef Mfma<T> M;
  typedef typename M::vec_t V;
  constexpr int ESZ = sizeof(T), VEC = 16 / ESZ;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  const int g = lane >> 4, l16 = lane & 15;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int kc = 4 * r + g;
    V a[FM];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int row = wm0 + 16 * i + l16;
      a[i] = *reinterpret_cast<const V *>(As + row * 128 + gd_swz_a(row, kc) * 16);
      if (TAIL) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) a[i][v] = kc * VEC + v < kvalid ? a[i][v] : T(0);
      }
    }
    if constexpr (BROW) {
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        const int kr = kc * VEC + v;
        T b[FN];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int byte = (wn0 + 16 * j + l16) * ESZ;
          b[j] = *reinterpret_cast<const T *>(
              Bs + kr * (BN * ESZ) + gd_swz_b<T>(kr, byte >> 4, BN * ESZ / 16) * 16 + (byte & 15));
          if (TAIL) b[j] = kr < kvalid ? b[j] : T(0);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = M::mma(a[i][v], b[j], acc[i][j]);
      }
    } else {
      V b[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        b[j] = *reinterpret_cast<const V *>(Bs + (kc * BN + wn0 + 16 * j + l16) * 16);
        if (TAIL) {
#pragma unroll
          for (int v = 0; v < VEC; ++v) b[j][v] = kc * VEC + v < kvalid ? b[j][v] : T(0);
        }
      }
#pragma unroll
      for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = M::mma(a[i][v], b[j][v], acc[i][j]);
    }
  }
}

template <typename T, int BM, int BN>
__device__ __forceinline__ void gd_store(const GTileRec<T> &t,
                                         const typename Mfma<T>::acc_t (&acc)[BM / 32][BN / 32],
                                         int wave, int lane) {
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  const int m0 = t.tm * BM + (wave >> 1) * WM, n0 = t.tn * BN + (wave & 1) * WN;
  if ((t.cls >> 4) & 1) Epilogue<T, true>::template store<FM, FN>(t.g, acc, m0, n0, lane);
  else Epilogue<T, false>::template store<FM, FN>(t.g, acc, m0, n0, lane);
}

// Tile record through the constant address space: the list is never written
// during the launch, so the uniform record loads become scalar loads, which
// do not count against the vector-memory counter the DMA ring waits on.
template <typename T>
__device__ __forceinline__ GTileRec<T> gd_record(const GTileRec<T> *tiles, int w) {
  typedef __attribute__((address_space(4))) const GTileRec<T> CRec;
  GTileRec<T> r;
  __builtin_memcpy(&r, (const GTileRec<T> *)&((const CRec *)tiles)[w], sizeof(r));
  return r;
}

// Load cursor of a workgroup: walks the same tiles as the compute side,
// NS-1 k-steps ahead, and remembers how many DMA instructions each issued
// but unconsumed step has (NS-1 of them).
// Tile of workgroup b in dealing round r: rounds alternate direction
// (b', then G-1-b'), so with the list in decreasing cost every workgroup gets
// a fair share of the expensive and of the cheap tiles.  b' numbers the
// workgroups XCD by XCD (the dispatcher places workgroup b on XCD b % 8), so
// each XCD takes a contiguous run of every round: the tiles of one problem,
// adjacent in the list, then share one L2.  Past the list: ntiles.
__device__ __forceinline__ int gd_deal(int r, int b, int G, int ntiles) {
  if ((int64_t)r * G >= ntiles) return ntiles;
  const int bx = xcd_remap(b, G);
  const int w = r * G + ((r & 1) ? G - 1 - bx : bx);
  return w < ntiles ? w : ntiles;
}

template <typename T>
struct GdLoader {
  const GTileRec<T> *tiles;
  int ntiles, G, lr, lw, lkt, li;
  GTileRec<T> L;
  GdSlots<T> sl;
  unsigned char *lds;
  int wave, lane;
  int q[kGdNS - 1];  // DMA counts of the issued, unconsumed steps, oldest first (0: none)

  // DMA instructions issued after the oldest unconsumed step.
  __device__ __forceinline__ int later() const {
    int n = 0;
#pragma unroll
    for (int i = 1; i < kGdNS - 1; ++i) n += q[i];
    return n;
  }
  // The oldest step was consumed; `cnt` is the step just issued.
  __device__ __forceinline__ void push(int cnt) {
#pragma unroll
    for (int i = 0; i < kGdNS - 2; ++i) q[i] = q[i + 1];
    q[kGdNS - 2] = cnt;
  }

  __device__ __forceinline__ void next_tile() {
    do {
      lw = gd_deal(++lr, (int)blockIdx.x, G, ntiles);
      if (lw < ntiles) L = gd_record(tiles, lw);
    } while (lw < ntiles && (L.cls & 15) == kScaleCls);
    if (lw < ntiles) {
      const int c = L.cls & 15;
      gd_setup<T>(sl, L.g, c, L.tm * gd_bm(c), L.tn * gd_bn(c), wave, lane, (L.cls >> 5) & 1,
                  (L.cls >> 6) & 1);
    }
  }
  // Issues the next k-step of the stream; returns its DMA count (0 if none).
  __device__ __forceinline__ int issue() {
    constexpr int BK = 128 / (int)sizeof(T);
    if (lw >= ntiles) return 0;
    const int cnt = gd_issue<T>(sl, L.g, L.cls, lkt * BK, lds + (li % kGdNS) * kGdStage,
                                wave, lane);
    ++li;
    if (++lkt * BK >= L.g.k) {
      lkt = 0;
      next_tile();
    }
    return cnt;
  }
};

// Waits until at most `n` (the DMA instructions of the steps issued after
// the current one) vector memory operations of this wave are outstanding:
// the current step has landed.  DMA instructions per step: A 8 / 4
// (4-byte, 64 / 32 rows) or 2 / 1 (16-byte) plus B 8 / 4 (4-byte, 64 / 32
// columns) or 2 / 1 (16-byte).
#define MG_GD_W1(N) \
  case N: gd_wait_vmcnt<N>(); break;
#define MG_GD_W4(N) MG_GD_W1(N) MG_GD_W1(N + 1) MG_GD_W1(N + 2) MG_GD_W1(N + 3)
#define MG_GD_W16(N) MG_GD_W4(N) MG_GD_W4(N + 4) MG_GD_W4(N + 8) MG_GD_W4(N + 12)
__device__ __forceinline__ void gd_wait_next(int n) {
  if constexpr (kGdNS <= 3) {  // one step behind the current one: at most 16
    switch (n) {  // the step counts that occur (a sum of one A and one B count)
      MG_GD_W1(16) MG_GD_W1(12) MG_GD_W1(10) MG_GD_W1(9) MG_GD_W1(8)
      MG_GD_W1(6) MG_GD_W1(5) MG_GD_W1(4) MG_GD_W1(3) MG_GD_W1(2)
      default: gd_wait_vmcnt<0>(); break;  // 0: wait for all
    }
  } else {
    switch (n) {
      MG_GD_W16(1)
      MG_GD_W16(17)
      MG_GD_W16(33)
      default: gd_wait_vmcnt<0>(); break;  // 0, or past the covered range: wait for all
    }
  }
}
#undef MG_GD_W16
#undef MG_GD_W4
#undef MG_GD_W1

// All k-steps of one tile of class (BM, BN), then its epilogue; `t` counts
// the workgroup's consumed steps (ring position).
template <typename T, int BM, int BN>
__device__ __forceinline__ void gd_run_tile(GdLoader<T> &ld, const GTileRec<T> &C, int &t) {
  typedef typename Mfma<T>::acc_t Acc;
  constexpr int BK = 128 / (int)sizeof(T);
  constexpr int FM = BM / 32, FN = BN / 32;
  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{};
  const int KT = (C.g.k + BK - 1) / BK;
  const bool brow = kGd16<T> && ((C.cls >> 6) & 1);
  for (int kt = 0; kt < KT; ++kt) {
    gd_wait_next(ld.later());
    __builtin_amdgcn_s_barrier();
    // the stage the loader refills next (consumed in the previous step)
    MG_LDS_POISON_STAGE(ld.lds + (ld.li % kGdNS) * kGdStage, kGdStage);
    // The ring's refill is issued at raised priority: the waves of the other
    // workgroups on this SIMD are mostly issuing MFMAs, and a refill held
    // behind them shortens the ring's lead (FP64 batch of 2000 problems:
    // 0.617 -> 0.58 ms; FP32 unchanged).
    __builtin_amdgcn_s_setprio(2);
    const int cnew = ld.issue();
    __builtin_amdgcn_s_setprio(0);
    const unsigned char *As = ld.lds + (t % kGdNS) * kGdStage;
    const unsigned char *Bs = As + kGdStageA;
    const int kvalid = C.g.k - kt * BK;
    if (brow) {  // always false for FP32: the row-major path is not built there
      if constexpr (kGd16<T>) {
        if (kvalid >= BK) gd_compute<T, BM, BN, false, true>(acc, As, Bs, ld.wave, ld.lane, kvalid);
        else gd_compute<T, BM, BN, true, true>(acc, As, Bs, ld.wave, ld.lane, kvalid);
      }
    } else {
      if (kvalid >= BK) gd_compute<T, BM, BN, false, false>(acc, As, Bs, ld.wave, ld.lane, kvalid);
      else gd_compute<T, BM, BN, true, false>(acc, As, Bs, ld.wave, ld.lane, kvalid);
    }
    ld.push(cnew);
    ++t;
  }
  gd_store<T, BM, BN>(C, acc, ld.wave, ld.lane);
}

template <typename T>
__global__ __launch_bounds__(kTileThreads, kGdMinBlocks) void grouped_dma_kernel(
    const GTileRec<T> *__restrict__ tiles, int ntiles) {
  extern __shared__ __align__(16) unsigned char lds[];
  GdLoader<T> ld;
  ld.tiles = tiles;
  ld.ntiles = ntiles;
  ld.G = (int)gridDim.x;
  ld.lds = lds;
  // wave index made uniform so LDS destinations (M0) are scalar arithmetic
  ld.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  ld.lane = threadIdx.x & 63;
  ld.lkt = 0;
  ld.li = 0;
  ld.lr = -1;
  MG_LDS_POISON_STAGE(lds, kGdNS * kGdStage);
  ld.next_tile();  // first tile with k-steps
#pragma unroll
  for (int i = 0; i < kGdNS - 1; ++i) ld.q[i] = ld.issue();

  int cr = 0, t = 0;
  for (int cw = gd_deal(0, blockIdx.x, ld.G, ntiles); cw < ntiles;
       cw = gd_deal(++cr, blockIdx.x, ld.G, ntiles)) {
    const GTileRec<T> C = gd_record(tiles, cw);
    const int c = C.cls & 15;
    if (c == kScaleCls) scale_tile<T>(C.g, C.tm * kScaleTile, C.tn * kScaleTile);
    else if (c == 0) gd_run_tile<T, 64, 64>(ld, C, t);
    else if (c == 1) gd_run_tile<T, 64, 32>(ld, C, t);
    else gd_run_tile<T, 32, 32>(ld, C, t);
  }
}

template <typename T>
size_t grouped_lds_bytes() {
  return (size_t)kGdNS * kGdStage;
}

int bucket_of(int64_t x) {
  int b = 0;
  while (b < kTuneEdges - 1 && x >= (int64_t)(32 << b)) ++b;
  return b;
}

}  // namespace

int tune_bucket(int64_t m, int64_t n, int64_t k) {
  return (bucket_of(m) * kTuneEdges + bucket_of(n)) * kTuneEdges + bucket_of(k);
}

int64_t tune_bucket_rep(int b) {  // representative extent of a 1-D bucket
  if (b == 0) return 22;                       // [1, 32)
  if (b == kTuneEdges - 1) return 16 << b;     // [512, ...)
  return (int64_t)std::lround(16.0 * std::sqrt(2.0) * (1 << b));  // geometric middle
}

int grouped_class_tile(int cls, int *bm, int *bn) {
  if (cls < 0 || cls >= kNumGroupedClasses) return MG_ERR_INVALID_ARG;
  *bm = kClsBM[cls];
  *bn = kClsBN[cls];
  return MG_OK;
}

// Heuristic class when no tuning table is given: the largest tile that does
// not waste more than a quarter of its area on padding.
int heuristic_class(int64_t m, int64_t n) {
  for (int c = 0; c < kNumGroupedClasses; ++c) {
    const double used = (double)(m * n);
    const double padded = (double)(round_up(m, kClsBM[c]) * round_up(n, kClsBN[c]));
    if (used >= 0.75 * padded) return c;
  }
  return kNumGroupedClasses - 1;
}

struct Plan {
  int dtype = MG_F64;
  int device = 0;
  int64_t count = 0;
  int ntiles = 0;
  int grid = 0;
  void *d_tiles = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mg_plan_stats stats{};
};

namespace {

template <typename T>
int build_t(int64_t count, const mg_problem *probs, const mg_tune_table *table, WorkList *out) {
  std::vector<GemmArgs<T>> hp((size_t)count);
  std::vector<GTileRec<T>> tiles;
  std::vector<double> cost;
  double flops = 0, bytes = 0;
  int64_t per_cls[kNumGroupedClasses + 1] = {0};
  for (int64_t i = 0; i < count; ++i) {
    const mg_problem &q = probs[i];
    GemmArgs<T> &g = hp[(size_t)i];
    g.A = static_cast<const T *>(q.A);
    g.B = static_cast<const T *>(q.B);
    g.C = static_cast<T *>(q.C);
    g.lda = q.lda;
    g.ldb = q.ldb;
    g.ldc = q.ldc;
    g.m = (int)q.m;
    g.n = (int)q.n;
    g.k = (int)q.k;
    g.alpha = (T)q.alpha;
    g.beta = (T)q.beta;
    if (q.m == 0 || q.n == 0) continue;
    if (q.k == 0 || q.alpha == 0.0) {
      const int tm = (int)ceil_div(q.m, kScaleTile), tn = (int)ceil_div(q.n, kScaleTile);
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          tiles.push_back(GTileRec<T>{g, a, b, kScaleCls, 0});
          cost.push_back((double)kScaleTile * kScaleTile);
        }
      per_cls[kNumGroupedClasses] += (int64_t)tm * tn;
      bytes += (double)q.m * q.n * sizeof(T) * (q.beta != 0.0 ? 2 : 1);
      continue;
    }
    int cls = table ? table->cls[tune_bucket(q.m, q.n, q.k)] : heuristic_class(q.m, q.n);
    if (cls < 0 || cls >= kNumGroupedClasses) cls = heuristic_class(q.m, q.n);
    const bool c_vec = vec_aligned(q.C, q.ldc, sizeof(T), Mfma<T>::VEC);
    const bool a_vec = vec_aligned(q.A, q.lda, sizeof(T), Mfma<T>::VEC);
    // 16-byte B loads (row-major B block) for FP64 only: FP32 reads that
    // layout one value per MFMA, four per 16-byte chunk, which measured
    // slower than its 4-byte loads into the k-interleaved block.
    const bool b_vec = sizeof(T) == 8 && vec_aligned(q.B, q.ldb, sizeof(T), Mfma<T>::VEC);
    const int bm = kClsBM[cls], bn = kClsBN[cls];
    const int tm = (int)ceil_div(q.m, bm), tn = (int)ceil_div(q.n, bn);
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        tiles.push_back(
            GTileRec<T>{g, a, b, cls | (c_vec ? 16 : 0) | (a_vec ? 32 : 0) | (b_vec ? 64 : 0), 0});
        // MFMA work of the padded tile plus its operand traffic (in FLOP-equivalents)
        cost.push_back(2.0 * bm * bn * (double)round_up(q.k, Mfma<T>::BK) +
                       16.0 * (bm + bn) * (double)q.k);
      }
    per_cls[cls] += (int64_t)tm * tn;
    flops += 2.0 * q.m * q.n * q.k;
    bytes += sizeof(T) * ((double)q.m * q.k + (double)q.k * q.n +
                          (double)q.m * q.n * (q.beta != 0.0 ? 2 : 1));
  }
  if (tiles.size() > (size_t)INT32_MAX) {
    set_error("too many tiles");
    return MG_ERR_INVALID_ARG;
  }
  // Longest-processing-time order: dealt round-robin to the workgroups, the
  // expensive tiles spread evenly and the cheap ones fill in at the end.
  std::vector<int> order(tiles.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  out->dtype = std::is_same<T, double>::value ? MG_F64 : MG_F32;
  out->tiles.resize(tiles.size() * sizeof(GTileRec<T>));
  GTileRec<T> *dst = reinterpret_cast<GTileRec<T> *>(out->tiles.data());
  for (size_t i = 0; i < order.size(); ++i) dst[i] = tiles[(size_t)order[i]];
  out->ntiles = (int)tiles.size();
  mg_plan_stats &st = out->stats;
  st = mg_plan_stats{};
  st.problems = count;
  st.tiles = out->ntiles;
  for (int c = 0; c < kNumGroupedClasses; ++c) st.tiles_per_class[c] = per_cls[c];
  st.scale_tiles = per_cls[kNumGroupedClasses];
  st.flops = flops;
  st.bytes = bytes;
  return MG_OK;
}

template <typename T>
int occupancy_t(int *cus, int *occ) {
  // Once per process (one device model), thread-safe through the static's
  // initialisation: CU count, the kernel's LDS limit, workgroups per CU.
  struct Occ {
    hipError_t err;
    const char *what;
    int cus, occ;
  };
  static const Occ o = [] {
    Occ r{hipSuccess, "", 0, 0};
    int dev = 0;
    const size_t lds = grouped_lds_bytes<T>();
    if ((r.err = hipGetDevice(&dev)) != hipSuccess) r.what = "hipGetDevice";
    else if ((r.err = hipDeviceGetAttribute(&r.cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
             hipSuccess)
      r.what = "hipDeviceGetAttribute";
    else if ((r.err = hipFuncSetAttribute(reinterpret_cast<const void *>(grouped_dma_kernel<T>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
             hipSuccess)
      r.what = "hipFuncSetAttribute";
    else if ((r.err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &r.occ, reinterpret_cast<const void *>(grouped_dma_kernel<T>), kTileThreads,
                  lds)) != hipSuccess)
      r.what = "hipOccupancyMaxActiveBlocksPerMultiprocessor";
    r.occ = std::max(1, r.occ);
    return r;
  }();
  if (o.err != hipSuccess) {
    set_error("%s failed: %s", o.what, hipGetErrorString(o.err));
    return MG_ERR_HIP;
  }
  *cus = o.cus;
  *occ = o.occ;
  return MG_OK;
}

template <typename T>
int launch_t(const void *d_tiles, int ntiles, int grid, hipStream_t s) {
  hipLaunchKernelGGL(grouped_dma_kernel<T>, dim3(grid), dim3(kTileThreads), grouped_lds_bytes<T>(), s,
                     static_cast<const GTileRec<T> *>(d_tiles), ntiles);
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

int launch_raw(Plan *p, hipStream_t s) {
  return launch_worklist(p->dtype, p->d_tiles, p->ntiles, p->grid, s);
}

}  // namespace

int build_worklist(int dtype, int64_t count, const mg_problem *probs, const mg_tune_table *table,
                   WorkList *out) {
  return dtype == MG_F64 ? build_t<double>(count, probs, table, out)
                         : build_t<float>(count, probs, table, out);
}

int grouped_grid(int dtype, int ntiles, int *grid, int *occupancy) {
  int cus = 0, occ = 0;
  int rc = dtype == MG_F64 ? occupancy_t<double>(&cus, &occ) : occupancy_t<float>(&cus, &occ);
  if (rc != MG_OK) return rc;
  *grid = std::max(1, std::min(ntiles, cus * occ));
  if (occupancy) *occupancy = occ;
  return MG_OK;
}

int launch_worklist(int dtype, const void *d_tiles, int ntiles, int grid, hipStream_t s) {
  if (ntiles == 0) return MG_OK;
  return dtype == MG_F64 ? launch_t<double>(d_tiles, ntiles, grid, s)
                         : launch_t<float>(d_tiles, ntiles, grid, s);
}

int plan_create(int dtype, int64_t count, const mg_problem *probs, const mg_tune_table *table,
                Plan **out) {
  WorkList wl;
  int rc = build_worklist(dtype, count, probs, table, &wl);
  if (rc != MG_OK) return rc;
  Plan *p = new Plan();
  p->dtype = dtype;
  p->count = count;
  p->ntiles = wl.ntiles;
  p->stats = wl.stats;
  int occ = 1;
  rc = grouped_grid(dtype, p->ntiles, &p->grid, &occ);
  if (rc == MG_OK) rc = (hipGetDevice(&p->device) == hipSuccess) ? MG_OK : MG_ERR_HIP;
  p->stats.workgroups = p->grid;
  p->stats.occupancy = occ;
  auto upload = [&](void **dst, const std::vector<unsigned char> &src) -> int {
    MG_HIP_TRY(hipMalloc(dst, std::max<size_t>(src.size(), 256)));
    if (!src.empty()) MG_HIP_TRY(hipMemcpy(*dst, src.data(), src.size(), hipMemcpyHostToDevice));
    return MG_OK;
  };
  if (rc == MG_OK) rc = upload(&p->d_tiles, wl.tiles);
  if (rc != MG_OK) {
    plan_destroy(p);
    return rc;
  }
  *out = p;
  return MG_OK;
}

int plan_launch(Plan *p, hipStream_t s, bool use_graph) {
  if (p->ntiles == 0) return MG_OK;
  if (!use_graph) return launch_raw(p, s);
  if (p->exec == nullptr) {
    // Capture the persistent launch once on a private stream.
    hipStream_t cap;
    MG_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      int rc = launch_raw(p, cap);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(cap, &g);
      if (rc != MG_OK || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cap);
        if (rc != MG_OK) return rc;
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e2));
        return MG_ERR_HIP;
      }
      p->graph = g;
      e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    }
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
      set_error("graph capture failed: %s", hipGetErrorString(e));
      return MG_ERR_HIP;
    }
    p->stats.graph = 1;
  }
  MG_HIP_TRY(hipGraphLaunch(p->exec, s));
  return MG_OK;
}

void plan_destroy(Plan *p) {
  if (p == nullptr) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  delete p;
}

const mg_plan_stats &plan_stats(const Plan *p) { return p->stats; }

// ---------------------------------------------------------------------------
// Batched launch without allocation: the work list lives in a fixed device
// array (one copy per GPU, held until the process ends) instead of memory
// the library allocates per call.

static __device__ __align__(256) unsigned char scratch[kNoAllocWorklistBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (the array's
// name is only a host-side stand-in).  Resolved once per device, with that
// device current.
int scratch_address(void **out) {
  int dev = 0;
  MG_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d the static work-list buffer supports", dev, kMaxDevices);
    return MG_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(e));
      return MG_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MG_OK;
}

}  // namespace

int gemm_batched_noalloc(int dtype, int64_t count, const mg_problem *probs, hipStream_t s) {
  // Host work list, reused by the calling thread (the copy below reads it
  // from pageable memory, which HIP stages before the call returns).
  thread_local WorkList wl;
  int rc = build_worklist(dtype, count, probs, nullptr, &wl);
  if (rc != MG_OK) return rc;
  if (wl.ntiles == 0) return MG_OK;
  if (wl.tiles.size() > kNoAllocWorklistBytes) {
    set_error("batch needs a %zu-byte work list (%d tiles); the static buffer holds %zu bytes",
              wl.tiles.size(), wl.ntiles, kNoAllocWorklistBytes);
    return MG_ERR_INVALID_ARG;
  }
  void *ptr = nullptr;
  if ((rc = scratch_address(&ptr)) != MG_OK) return rc;
  int grid = 1;
  if ((rc = grouped_grid(dtype, wl.ntiles, &grid, nullptr)) != MG_OK) return rc;
  MG_HIP_TRY(hipMemcpyAsync(ptr, wl.tiles.data(), wl.tiles.size(), hipMemcpyHostToDevice, s));
  return launch_worklist(dtype, ptr, wl.ntiles, grid, s);
}

}  // namespace mg

namespace mg {

namespace {

constexpr int kTuneMinProblems = 48;
constexpr int kTuneMaxProblems = 4096;
constexpr int kTuneWavesOfTiles = 4;          // tiles per workgroup slot when timing
constexpr int64_t kTuneOperandElems = 1 << 24;  // per operand scratch (A, B)

// Problems per bucket: enough that even the largest tile class gives every
// workgroup slot several tiles, so a class is judged by its throughput in a
// full batch rather than by the parallelism a few problems expose.
int64_t tune_count(int64_t m, int64_t n, int grid) {
  const int64_t t0 = ceil_div(m, kClsBM[0]) * ceil_div(n, kClsBN[0]);
  const int64_t want = ceil_div((int64_t)kTuneWavesOfTiles * grid, t0);
  return std::min<int64_t>(kTuneMaxProblems, std::max<int64_t>(kTuneMinProblems, want));
}

int time_plan(Plan *p, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *ms) {
  int rc = plan_launch(p, s, false);  // warm-up
  if (rc != MG_OK) return rc;
  MG_HIP_TRY(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) {
    rc = plan_launch(p, s, false);
    if (rc != MG_OK) return rc;
  }
  MG_HIP_TRY(hipEventRecord(e1, s));
  MG_HIP_TRY(hipEventSynchronize(e1));
  MG_HIP_TRY(hipEventElapsedTime(ms, e0, e1));
  return MG_OK;
}

}  // namespace

int autotune(int dtype, int reps, hipStream_t s, mg_tune_table *out) {
  const size_t esz = dtype == MG_F64 ? 8 : 4;
  int grid = 0;
  int rc = grouped_grid(dtype, INT32_MAX, &grid, nullptr);
  if (rc != MG_OK) return rc;
  // C needs a private region per problem; A and B are carved round-robin
  // from fixed scratch so that consecutive problems read different memory.
  int64_t c_elems = 0;
  for (int b = 0; b < kTuneEdges; ++b)
    for (int c = 0; c < kTuneEdges; ++c) {
      const int64_t m = tune_bucket_rep(b), n = tune_bucket_rep(c);
      c_elems = std::max(c_elems, tune_count(m, n, grid) * round_up(m * n, 64));
    }
  void *dA = nullptr, *dB = nullptr, *dC = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (dA) (void)hipFree(dA);
    if (dB) (void)hipFree(dB);
    if (dC) (void)hipFree(dC);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const size_t op_bytes = (size_t)kTuneOperandElems * esz;
  if (hipMalloc(&dA, op_bytes) != hipSuccess || hipMalloc(&dB, op_bytes) != hipSuccess ||
      hipMalloc(&dC, (size_t)c_elems * esz) != hipSuccess) {
    cleanup();
    set_error("autotune: scratch allocation failed");
    return MG_ERR_NO_MEMORY;
  }
  if (hipMemset(dA, 0, op_bytes) != hipSuccess || hipMemset(dB, 0, op_bytes) != hipSuccess ||
      hipMemset(dC, 0, (size_t)c_elems * esz) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    set_error("autotune: scratch setup failed");
    return MG_ERR_HIP;
  }
  out->dtype = dtype;
  std::vector<mg_problem> probs;
  mg_tune_table forced;
  for (int bm = 0; bm < kTuneEdges && rc == MG_OK; ++bm)
    for (int bn = 0; bn < kTuneEdges && rc == MG_OK; ++bn)
      for (int bk = 0; bk < kTuneEdges && rc == MG_OK; ++bk) {
        const int64_t m = tune_bucket_rep(bm), n = tune_bucket_rep(bn), k = tune_bucket_rep(bk);
        const int64_t count = tune_count(m, n, grid);
        const int64_t a_sz = round_up(m * k, 64), b_sz = round_up(k * n, 64);
        const int64_t c_sz = round_up(m * n, 64);
        probs.assign((size_t)count, mg_problem{});
        int64_t oa = 0, ob = 0;
        for (int64_t i = 0; i < count; ++i) {
          if (oa + a_sz > kTuneOperandElems) oa = 0;
          if (ob + b_sz > kTuneOperandElems) ob = 0;
          mg_problem &q = probs[(size_t)i];
          q.m = m;
          q.n = n;
          q.k = k;
          q.alpha = 1.0;
          q.beta = 1.0;
          q.A = static_cast<char *>(dA) + (size_t)oa * esz;
          q.lda = k;
          q.B = static_cast<char *>(dB) + (size_t)ob * esz;
          q.ldb = n;
          q.C = static_cast<char *>(dC) + (size_t)(i * c_sz) * esz;
          q.ldc = n;
          oa += a_sz;
          ob += b_sz;
        }
        float best = 0;
        int best_cls = heuristic_class(m, n);
        for (int c = 0; c < kNumGroupedClasses && rc == MG_OK; ++c) {
          forced.dtype = dtype;
          for (int b = 0; b < MG_TUNE_BUCKETS; ++b) forced.cls[b] = c;
          Plan *p = nullptr;
          rc = plan_create(dtype, count, probs.data(), &forced, &p);
          if (rc != MG_OK) break;
          float ms = 0;
          rc = time_plan(p, reps, s, e0, e1, &ms);
          plan_destroy(p);
          if (rc == MG_OK && (c == 0 || ms < best)) {
            best = ms;
            best_cls = c;
          }
        }
        out->cls[(bm * kTuneEdges + bn) * kTuneEdges + bk] = best_cls;
      }
  cleanup();
  return rc;
}

}  // namespace mg
