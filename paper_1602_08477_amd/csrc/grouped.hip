// Batched uneven GEMMs in one persistent launch.
//
// A plan turns a list of independent problems C_i <- alpha_i A_i B_i +
// beta_i C_i into a device work list of macro-tiles (each record carries its
// problem's arguments, tile coordinates and a tile class from the tuning
// table), sorted longest first.  One persistent kernel of (CUs x occupancy)
// workgroups walks the list round-robin (workgroup b takes tiles b, b+G,
// b+2G, ...: with the list in decreasing cost this deals the expensive tiles
// out evenly) and runs the same per-tile code as the single-problem kernel,
// so a problem's result does not depend on what else is in the batch.  Each
// workgroup loads its next record while it computes the current tile.  The
// launch is captured once in a HIP graph and replayed.
//
// In the paper's terms (Section 3.2): blocks are independent and are never
// synchronised with each other; they share nothing but the read-only list.
#include "grouped.h"

#include <algorithm>
#include <cmath>
#include <cstring>
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
  int cls;  // class | (vec_ok << 4)
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

template <typename T>
__device__ __forceinline__ void run_tile(const GTileRec<T> &t, T *smem) {
  const bool vec = (t.cls >> 4) & 1;
  switch (t.cls & 15) {
    case 0:
      if (vec) gemm_tile<T, 64, 64, true>(t.g, t.tm * 64, t.tn * 64, smem);
      else gemm_tile<T, 64, 64, false>(t.g, t.tm * 64, t.tn * 64, smem);
      break;
    case 1:
      if (vec) gemm_tile<T, 64, 32, true>(t.g, t.tm * 64, t.tn * 32, smem);
      else gemm_tile<T, 64, 32, false>(t.g, t.tm * 64, t.tn * 32, smem);
      break;
    case 2:
      if (vec) gemm_tile<T, 32, 32, true>(t.g, t.tm * 32, t.tn * 32, smem);
      else gemm_tile<T, 32, 32, false>(t.g, t.tm * 32, t.tn * 32, smem);
      break;
    default:
      scale_tile<T>(t.g, t.tm * kScaleTile, t.tn * kScaleTile);
      break;
  }
}

// Persistent loop over tiles blockIdx.x, +gridDim.x, ...; the next record is
// loaded (uniform, scalar loads) before the current tile is computed.
template <typename T>
__global__ __launch_bounds__(kTileThreads, 3) void grouped_kernel(
    const GTileRec<T> *__restrict__ tiles, int ntiles) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *smem = reinterpret_cast<T *>(lds_raw);
  int w = blockIdx.x;
  if (w >= ntiles) return;
  GTileRec<T> cur = tiles[w];
  for (;;) {
    const int nw = w + (int)gridDim.x;
    GTileRec<T> nxt = cur;
    if (nw < ntiles) nxt = tiles[nw];
    run_tile<T>(cur, smem);
    if (nw >= ntiles) break;
    __syncthreads();  // LDS of this tile fully consumed before the next one
    w = nw;
    cur = nxt;
  }
}

template <typename T>
size_t grouped_lds_bytes() {
  return std::max({TileShape<T, 64, 64>::LDS_BYTES, TileShape<T, 64, 32>::LDS_BYTES,
                   TileShape<T, 32, 32>::LDS_BYTES});
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
    constexpr int VEC = Mfma<T>::VEC;
    const bool vec = vec_aligned(q.A, q.lda, sizeof(T), VEC) &&
                     vec_aligned(q.B, q.ldb, sizeof(T), VEC) &&
                     vec_aligned(q.C, q.ldc, sizeof(T), VEC);
    const int bm = kClsBM[cls], bn = kClsBN[cls];
    const int tm = (int)ceil_div(q.m, bm), tn = (int)ceil_div(q.n, bn);
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        tiles.push_back(GTileRec<T>{g, a, b, cls | (vec ? 16 : 0), 0});
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
  static int s_cus = 0, s_occ = 0;  // per process: one device model
  if (s_occ == 0) {
    int dev = 0;
    MG_HIP_TRY(hipGetDevice(&dev));
    MG_HIP_TRY(hipDeviceGetAttribute(&s_cus, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t lds = grouped_lds_bytes<T>();
    MG_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(grouped_kernel<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int o = 0;
    MG_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &o, reinterpret_cast<const void *>(grouped_kernel<T>), kTileThreads, lds));
    s_occ = std::max(1, o);
  }
  *cus = s_cus;
  *occ = s_occ;
  return MG_OK;
}

template <typename T>
int launch_t(const void *d_tiles, int ntiles, int grid, hipStream_t s) {
  hipLaunchKernelGGL(grouped_kernel<T>, dim3(grid), dim3(kTileThreads), grouped_lds_bytes<T>(), s,
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
    // Capture reset + persistent kernel once on a private stream.
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

}  // namespace mg

namespace mg {

namespace {

constexpr int kTuneMaxExtent = 512;
constexpr int kTuneProblems = 48;

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
  const size_t mat = (size_t)kTuneMaxExtent * kTuneMaxExtent * esz;
  void *dA = nullptr, *dB = nullptr, *dC = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MG_OK;
  auto cleanup = [&]() {
    if (dA) (void)hipFree(dA);
    if (dB) (void)hipFree(dB);
    if (dC) (void)hipFree(dC);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&dA, mat) != hipSuccess || hipMalloc(&dB, mat) != hipSuccess ||
      hipMalloc(&dC, mat * kTuneProblems) != hipSuccess) {
    cleanup();
    set_error("autotune: scratch allocation failed");
    return MG_ERR_NO_MEMORY;
  }
  if (hipMemset(dA, 0, mat) != hipSuccess || hipMemset(dB, 0, mat) != hipSuccess ||
      hipMemset(dC, 0, mat * kTuneProblems) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    set_error("autotune: scratch setup failed");
    return MG_ERR_HIP;
  }
  out->dtype = dtype;
  std::vector<mg_problem> probs(kTuneProblems);
  mg_tune_table forced;
  for (int bm = 0; bm < kTuneEdges && rc == MG_OK; ++bm)
    for (int bn = 0; bn < kTuneEdges && rc == MG_OK; ++bn)
      for (int bk = 0; bk < kTuneEdges && rc == MG_OK; ++bk) {
        const int64_t m = tune_bucket_rep(bm), n = tune_bucket_rep(bn), k = tune_bucket_rep(bk);
        for (int i = 0; i < kTuneProblems; ++i) {
          mg_problem &q = probs[(size_t)i];
          q.m = m;
          q.n = n;
          q.k = k;
          q.alpha = 1.0;
          q.beta = 1.0;
          q.A = dA;
          q.lda = k;
          q.B = dB;
          q.ldb = n;
          q.C = static_cast<char *>(dC) + (size_t)i * mat;
          q.ldc = n;
        }
        float best = 0;
        int best_cls = heuristic_class(m, n);
        for (int c = 0; c < kNumGroupedClasses && rc == MG_OK; ++c) {
          forced.dtype = dtype;
          for (int b = 0; b < MG_TUNE_BUCKETS; ++b) forced.cls[b] = c;
          Plan *p = nullptr;
          rc = plan_create(dtype, kTuneProblems, probs.data(), &forced, &p);
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
