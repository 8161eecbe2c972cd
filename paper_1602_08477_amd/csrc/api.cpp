// extern "C" boundary of libmg: argument validation, error reporting and
// dispatch to the kernels.  Nothing is enqueued when validation fails.
#include <cstdlib>
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <list>
#include <mutex>
#include <utility>
#include <vector>

#include "axpy.h"
#include "common.h"
#include "gemm_native.h"
#include "grouped.h"
#include "split.h"

namespace mg {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

int validate_problem(const char *what, int64_t m, int64_t n, int64_t k, double alpha,
                     const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
                     const void *C, int64_t ldc, int64_t esz) {
  return validate_problem_op(what, false, false, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                             esz);
}

int validate_problem_op(const char *what, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                        double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                        double beta, const void *C, int64_t ldc, int64_t esz) {
  (void)beta;
  if (m < 0 || n < 0 || k < 0) {
    set_error("%s: negative extent (m=%lld n=%lld k=%lld)", what, (long long)m, (long long)n,
              (long long)k);
    return MG_ERR_INVALID_ARG;
  }
  // Extents index with 32-bit ints inside tiles; pitches and offsets are 64-bit.
  const int64_t lim = (int64_t)1 << 30;
  if (m >= lim || n >= lim || k >= lim) {
    set_error("%s: extent too large (limit 2^30)", what);
    return MG_ERR_INVALID_ARG;
  }
  if (m == 0 || n == 0) return MG_OK;
  if (C == nullptr) {
    set_error("%s: C is NULL", what);
    return MG_ERR_INVALID_ARG;
  }
  if (ldc < n) {
    set_error("%s: ldc=%lld < n=%lld", what, (long long)ldc, (long long)n);
    return MG_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(C) % (uintptr_t)esz) {
    set_error("%s: C not aligned to its element size", what);
    return MG_ERR_INVALID_ARG;
  }
  const int64_t big = (int64_t)1 << 62;
  if ((m - 1) > big / ldc) {
    set_error("%s: C extent overflows", what);
    return MG_ERR_INVALID_ARG;
  }
  const bool reads_ab = k > 0 && alpha != 0.0;
  if (!reads_ab) return MG_OK;
  if (A == nullptr || B == nullptr) {
    set_error("%s: A or B is NULL", what);
    return MG_ERR_INVALID_ARG;
  }
  // Stored shapes: A is m x k (k x m when transposed), B is k x n (n x k).
  const int64_t a_rows = ta ? k : m, a_cols = ta ? m : k;
  const int64_t b_rows = tb ? n : k, b_cols = tb ? k : n;
  if (lda < a_cols) {
    set_error("%s: lda=%lld < %s=%lld", what, (long long)lda, ta ? "m" : "k", (long long)a_cols);
    return MG_ERR_INVALID_ARG;
  }
  if (ldb < b_cols) {
    set_error("%s: ldb=%lld < %s=%lld", what, (long long)ldb, tb ? "k" : "n", (long long)b_cols);
    return MG_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(A) % (uintptr_t)esz ||
      reinterpret_cast<uintptr_t>(B) % (uintptr_t)esz) {
    set_error("%s: A or B not aligned to its element size", what);
    return MG_ERR_INVALID_ARG;
  }
  if ((a_rows - 1) > big / lda || (b_rows - 1) > big / ldb) {
    set_error("%s: A or B extent overflows", what);
    return MG_ERR_INVALID_ARG;
  }
  if (spans_overlap(C, m, n, ldc, A, a_rows, a_cols, lda, esz) ||
      spans_overlap(C, m, n, ldc, B, b_rows, b_cols, ldb, esz)) {
    set_error("%s: C overlaps A or B", what);
    return MG_ERR_INVALID_ARG;
  }
  return MG_OK;
}

static int64_t esize(int dtype) { return dtype == MG_F64 ? 8 : dtype == MG_F32 ? 4 : 0; }

// Validates every problem of a batch and that no output overlaps another
// problem's output or any operand.
int validate_batch(int dtype, int64_t count, const mg_problem *probs) {
  const int64_t es = esize(dtype);
  if (es == 0) {
    set_error("unknown dtype %d", dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (count < 0 || (count > 0 && probs == nullptr) || count > ((int64_t)1 << 30)) {
    set_error("bad problem count %lld or NULL problem array", (long long)count);
    return MG_ERR_INVALID_ARG;
  }
  char what[64];
  struct Span {
    uintptr_t lo, hi;
    int64_t idx;
  };
  std::vector<Span> cs, ops;
  for (int64_t i = 0; i < count; ++i) {
    const mg_problem &q = probs[i];
    snprintf(what, sizeof(what), "problem %lld", (long long)i);
    int rc = validate_problem(what, q.m, q.n, q.k, q.alpha, q.A, q.lda, q.B, q.ldb, q.beta, q.C,
                              q.ldc, es);
    if (rc != MG_OK) return rc;
    if (q.m == 0 || q.n == 0) continue;
    Span c;
    byte_span(q.C, q.m, q.n, q.ldc, es, c.lo, c.hi);
    c.idx = i;
    cs.push_back(c);
    if (q.k > 0 && q.alpha != 0.0) {
      Span a, b;
      byte_span(q.A, q.m, q.k, q.lda, es, a.lo, a.hi);
      byte_span(q.B, q.k, q.n, q.ldb, es, b.lo, b.hi);
      a.idx = b.idx = i;
      ops.push_back(a);
      ops.push_back(b);
    }
  }
  std::sort(cs.begin(), cs.end(), [](const Span &x, const Span &y) { return x.lo < y.lo; });
  for (size_t i = 1; i < cs.size(); ++i)
    if (cs[i].lo < cs[i - 1].hi) {
      set_error("outputs of problems %lld and %lld overlap", (long long)cs[i - 1].idx,
                (long long)cs[i].idx);
      return MG_ERR_INVALID_ARG;
    }
  for (const Span &o : ops) {
    // last output starting below o.hi; outputs are disjoint, so ends are sorted too
    auto it = std::lower_bound(cs.begin(), cs.end(), o.hi,
                               [](const Span &x, uintptr_t v) { return x.lo < v; });
    if (it != cs.begin() && std::prev(it)->hi > o.lo) {
      set_error("an operand of problem %lld overlaps the output of problem %lld",
                (long long)o.idx, (long long)std::prev(it)->idx);
      return MG_ERR_INVALID_ARG;
    }
  }
  return MG_OK;
}

// One-shot batches: plans whose device memory is released once the event
// recorded after their launch has completed.
std::mutex g_deferred_mu;
std::vector<std::pair<Plan *, hipEvent_t>> g_deferred;

// One-shot batches whose problem set repeats replay the graph of the plan
// built the first time.  The last kPlanCacheSize distinct sets are kept,
// matched on device, dtype and every descriptor byte for byte: the work list
// holds only pointers, extents and scalars, so a replay reads the operands'
// current contents.  An evicted plan is freed once its last launch has
// completed (deferred like a one-shot plan).
struct CachedBatch {
  int device = 0, dtype = 0;
  uint64_t hash = 0;
  std::vector<mg_problem> probs;
  Plan *plan = nullptr;
  hipEvent_t last = nullptr;  // recorded after the latest launch of the plan
};
constexpr size_t kPlanCacheSize = 8;
std::mutex g_cache_mu;
std::list<CachedBatch> g_cache;  // most recently used first
int64_t g_cache_hits = 0, g_cache_misses = 0;

// Word-wise multiply-xor hash of the descriptors (a mg_problem is eleven
// 8-byte fields, no padding).
uint64_t hash_problems(int dtype, int64_t count, const mg_problem *p) {
  static_assert(sizeof(mg_problem) == 11 * sizeof(uint64_t), "descriptor without padding");
  uint64_t h = 0x9e3779b97f4a7c15ull ^ (uint64_t)dtype ^ ((uint64_t)count << 8);
  const size_t words = (size_t)count * (sizeof(mg_problem) / sizeof(uint64_t));
  for (size_t i = 0; i < words; ++i) {
    uint64_t w;
    std::memcpy(&w, reinterpret_cast<const unsigned char *>(p) + i * 8, 8);
    h = (h ^ w) * 0xff51afd7ed558ccdull;
    h ^= h >> 29;
  }
  return h;
}

void reap_deferred(bool wait) {
  std::lock_guard<std::mutex> lk(g_deferred_mu);
  std::vector<std::pair<Plan *, hipEvent_t>> keep;
  for (auto &pe : g_deferred) {
    if (wait) (void)hipEventSynchronize(pe.second);
    if (hipEventQuery(pe.second) == hipSuccess) {
      plan_destroy(pe.first);
      (void)hipEventDestroy(pe.second);
    } else {
      keep.push_back(pe);
    }
  }
  g_deferred.swap(keep);
}

}  // namespace mg

using namespace mg;

extern "C" {

const char *mg_last_error(void) { return g_err; }

int mg_version(void) { return 10100; }

int mg_build_flags(void) {
#ifdef MG_LDS_POISON
  return MG_BUILD_LDS_POISON;
#else
  return 0;
#endif
}

int mg_num_tile_cfgs(void) { return num_tile_cfgs(); }

int mg_tile_cfg_info(int dtype, int cfg, int *bm, int *bn, int *bk, int *threads) {
  clear_error();
  return tile_cfg_info(dtype, cfg, bm, bn, bk, threads);
}

int mg_pick_tile_cfg(int dtype, int64_t m, int64_t n, int64_t k) {
  return pick_tile_cfg(dtype, m, n, k);
}

int mg_gemm_cfg(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
                int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
                void *stream) {
  clear_error();
  const int64_t es = esize(dtype);
  if (es == 0) {
    set_error("unknown dtype %d", dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (cfg < 0 || cfg >= num_tile_cfgs()) {
    set_error("unknown tile cfg %d", cfg);
    return MG_ERR_INVALID_ARG;
  }
  int rc = validate_problem("gemm", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, es);
  if (rc != MG_OK) return rc;
  return gemm_native(dtype, cfg, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                     static_cast<hipStream_t>(stream));
}

int mg_gemm_ex(int dtype, int cfg, int transa, int transb, int64_t m, int64_t n, int64_t k,
               double alpha, const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
               void *C, int64_t ldc, void *stream) {
  clear_error();
  const int64_t es = esize(dtype);
  if (es == 0) {
    set_error("unknown dtype %d", dtype);
    return MG_ERR_INVALID_ARG;
  }
  if ((transa != 0 && transa != 1) || (transb != 0 && transb != 1)) {
    set_error("transa/transb must be 0 or 1 (got %d, %d)", transa, transb);
    return MG_ERR_INVALID_ARG;
  }
  if (cfg < -1 || cfg >= num_tile_cfgs()) {
    set_error("unknown tile cfg %d", cfg);
    return MG_ERR_INVALID_ARG;
  }
  int rc = validate_problem_op("gemm_ex", transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C,
                               ldc, es);
  if (rc != MG_OK) return rc;
  if (cfg < 0) cfg = pick_tile_cfg(dtype, m, n, k);
  return gemm_native_op(dtype, cfg, transa, transb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                        static_cast<hipStream_t>(stream));
}

int mg_daxpy(int64_t n, double alpha, const double *x, int64_t incx, double *y, int64_t incy,
             void *stream) {
  clear_error();
  if (n < 0) {
    set_error("daxpy: negative n=%lld", (long long)n);
    return MG_ERR_INVALID_ARG;
  }
  if (incx < 1 || incy < 1) {
    set_error("daxpy: increments must be >= 1 (incx=%lld incy=%lld)", (long long)incx,
              (long long)incy);
    return MG_ERR_INVALID_ARG;
  }
  if (n == 0 || alpha == 0.0) return MG_OK;
  if (x == nullptr || y == nullptr) {
    set_error("daxpy: x or y is NULL");
    return MG_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(x) % 8 || reinterpret_cast<uintptr_t>(y) % 8) {
    set_error("daxpy: x or y not aligned to 8 bytes");
    return MG_ERR_INVALID_ARG;
  }
  const int64_t big = (int64_t)1 << 59;
  if (n - 1 > big / incx || n - 1 > big / incy) {
    set_error("daxpy: vector extent overflows");
    return MG_ERR_INVALID_ARG;
  }
  // y may be x itself (same increment: each element reads and writes only
  // itself); any other overlap would race.
  if (!(x == y && incx == incy) && spans_overlap(x, 1, (n - 1) * incx + 1, 1, y, 1,
                                                 (n - 1) * incy + 1, 1, 8)) {
    set_error("daxpy: x and y overlap");
    return MG_ERR_INVALID_ARG;
  }
  return axpy_f64(n, alpha, x, incx, y, incy, static_cast<hipStream_t>(stream));
}

int mg_gemm(int dtype, int algo, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
            int64_t lda, const void *B, int64_t ldb, double beta, void *C, int64_t ldc,
            void *stream) {
  clear_error();
  const int64_t es = esize(dtype);
  if (es == 0) {
    set_error("unknown dtype %d", dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (algo != MG_NATIVE && algo != MG_SPLIT_I8 && algo != MG_SPLIT_BF16) {
    set_error("unknown algo %d", algo);
    return MG_ERR_INVALID_ARG;
  }
  if (algo != MG_NATIVE && dtype != MG_F64) {
    set_error("split algorithms take FP64 operands");
    return MG_ERR_UNSUPPORTED;
  }
  int rc = validate_problem("gemm", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, es);
  if (rc != MG_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (algo == MG_NATIVE)
    return gemm_native(dtype, pick_tile_cfg(dtype, m, n, k), m, n, k, alpha, A, lda, B, ldb,
                       beta, C, ldc, s);
  return gemm_split_pooled(algo, split_default_slices(algo), m, n, k, alpha,
                           static_cast<const double *>(A), lda, static_cast<const double *>(B),
                           ldb, beta, static_cast<double *>(C), ldc, s);
}

int mg_split_default_slices(int algo) {
  clear_error();
  if (algo != MG_SPLIT_I8 && algo != MG_SPLIT_BF16) {
    set_error("not a split algorithm: %d", algo);
    return MG_ERR_INVALID_ARG;
  }
  return split_default_slices(algo);
}

int mg_split_layout_query(int algo, int slices, int64_t m, int64_t n, int64_t k,
                          mg_split_layout *out) {
  clear_error();
  if (out == nullptr) {
    set_error("out is NULL");
    return MG_ERR_INVALID_ARG;
  }
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  out->mp = L.mp;
  out->np = L.np;
  out->kp = L.kp;
  out->elem_bytes = L.elem_bytes;
  out->e_off = L.e_off;
  out->f_off = L.f_off;
  out->a_off = L.a_off;
  out->b_off = L.b_off;
  out->p_off = L.p_off;
  out->total_bytes = L.total;
  return MG_OK;
}

int mg_split_prepare(int algo, int slices, int64_t m, int64_t n, int64_t k, const double *A,
                     int64_t lda, const double *B, int64_t ldb, void *workspace,
                     int64_t workspace_bytes, void *stream) {
  clear_error();
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  // Validate A and B as operands of an m x n product (C is not touched).
  double dummy = 0.0;
  rc = validate_problem("split_prepare", std::max<int64_t>(m, 1), std::max<int64_t>(n, 1), k, 1.0,
                        A, lda, B, ldb, 0.0, &dummy, std::max<int64_t>(n, 1), 8);
  if (rc != MG_OK) return rc;
  if (workspace == nullptr || workspace_bytes < L.total) {
    set_error("split workspace too small: need %lld bytes", (long long)L.total);
    return MG_ERR_INVALID_ARG;
  }
  if (k > 0 && (A == nullptr || B == nullptr)) {
    set_error("A or B is NULL");
    return MG_ERR_INVALID_ARG;
  }
  return split_prepare(algo, slices, m, n, k, A, lda, B, ldb, workspace,
                       static_cast<hipStream_t>(stream));
}

int mg_split_num_cfgs(void) { return split_num_cfgs(); }

int mg_release_cached_memory(void) {
  clear_error();
  return release_workspace_pools();
}

int mg_gemm_split_cfg(int algo, int slices, int cfg, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double beta, double *C, int64_t ldc, void *workspace,
                      int64_t workspace_bytes, void *stream) {
  clear_error();
  if (cfg < -1 || cfg >= split_num_cfgs()) {
    set_error("unknown split cfg %d", cfg);
    return MG_ERR_INVALID_ARG;
  }
  SplitLayout L;
  int rc = split_layout(algo, slices, m, n, k, &L);
  if (rc != MG_OK) return rc;
  rc = validate_problem("gemm_split", m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, 8);
  if (rc != MG_OK) return rc;
  const bool reads_ab = k > 0 && alpha != 0.0;
  if (workspace != nullptr && workspace_bytes > 0 && reads_ab && m > 0 && n > 0) {
    const uintptr_t w0 = reinterpret_cast<uintptr_t>(workspace);
    const uintptr_t w1 = w0 + (uintptr_t)workspace_bytes;
    uintptr_t lo, hi;
    bool bad = false;
    byte_span(C, m, n, ldc, 8, lo, hi);
    bad |= lo < w1 && w0 < hi;
    byte_span(A, m, k, lda, 8, lo, hi);
    bad |= lo < w1 && w0 < hi;
    byte_span(B, k, n, ldb, 8, lo, hi);
    bad |= lo < w1 && w0 < hi;
    if (bad) {
      set_error("workspace overlaps A, B or C");
      return MG_ERR_INVALID_ARG;
    }
  }
  return gemm_split(algo, slices, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, workspace,
                    workspace_bytes, static_cast<hipStream_t>(stream), cfg);
}

int mg_gemm_split(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                  double *C, int64_t ldc, void *workspace, int64_t workspace_bytes,
                  void *stream) {
  return mg_gemm_split_cfg(algo, slices, -1, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc,
                           workspace, workspace_bytes, stream);
}

int mg_grouped_class_info(int cls, int *bm, int *bn) {
  clear_error();
  int a = 0, b = 0;
  if (grouped_class_tile(cls, &a, &b) != MG_OK) {
    set_error("unknown tile class %d", cls);
    return MG_ERR_INVALID_ARG;
  }
  if (bm) *bm = a;
  if (bn) *bn = b;
  return MG_OK;
}

int mg_tune_bucket(int64_t m, int64_t n, int64_t k) { return tune_bucket(m, n, k); }

int mg_tune_default(int dtype, mg_tune_table *out) {
  clear_error();
  if (out == nullptr || esize(dtype) == 0) {
    set_error("bad dtype or NULL table");
    return MG_ERR_INVALID_ARG;
  }
  out->dtype = dtype;
  for (int bm = 0; bm < kTuneEdges; ++bm)
    for (int bn = 0; bn < kTuneEdges; ++bn)
      for (int bk = 0; bk < kTuneEdges; ++bk)
        out->cls[(bm * kTuneEdges + bn) * kTuneEdges + bk] =
            heuristic_class(tune_bucket_rep(bm), tune_bucket_rep(bn));
  return MG_OK;
}

int mg_autotune(int dtype, int reps, void *stream, mg_tune_table *out) {
  clear_error();
  if (out == nullptr || esize(dtype) == 0 || reps < 1) {
    set_error("bad dtype, reps or NULL table");
    return MG_ERR_INVALID_ARG;
  }
  return autotune_cached(dtype, reps, std::getenv("MG_AUTOTUNE_CACHE"),
                         static_cast<hipStream_t>(stream), out, nullptr);
}

int mg_autotune_cached(int dtype, int reps, const char *cache_path, void *stream,
                       mg_tune_table *out, int *from_cache) {
  clear_error();
  if (out == nullptr || esize(dtype) == 0 || reps < 1) {
    set_error("bad dtype, reps or NULL table");
    return MG_ERR_INVALID_ARG;
  }
  return autotune_cached(dtype, reps, cache_path, static_cast<hipStream_t>(stream), out,
                         from_cache);
}

int mg_plan_create(int dtype, int64_t count, const mg_problem *probs, const mg_tune_table *table,
                   mg_plan **out) {
  clear_error();
  if (out == nullptr) {
    set_error("out is NULL");
    return MG_ERR_INVALID_ARG;
  }
  *out = nullptr;
  int rc = validate_batch(dtype, count, probs);
  if (rc != MG_OK) return rc;
  if (table != nullptr && table->dtype != dtype) {
    set_error("tuning table is for dtype %d, plan is %d", table->dtype, dtype);
    return MG_ERR_INVALID_ARG;
  }
  Plan *p = nullptr;
  rc = plan_create(dtype, count, probs, table, &p);
  if (rc != MG_OK) return rc;
  *out = reinterpret_cast<mg_plan *>(p);
  return MG_OK;
}

int mg_plan_launch(mg_plan *plan, void *stream) {
  clear_error();
  if (plan == nullptr) {
    set_error("plan is NULL");
    return MG_ERR_INVALID_ARG;
  }
  return plan_launch(reinterpret_cast<Plan *>(plan), static_cast<hipStream_t>(stream), true);
}

int mg_plan_launch_direct(mg_plan *plan, void *stream) {
  clear_error();
  if (plan == nullptr) {
    set_error("plan is NULL");
    return MG_ERR_INVALID_ARG;
  }
  return plan_launch(reinterpret_cast<Plan *>(plan), static_cast<hipStream_t>(stream), false);
}

int mg_plan_get_stats(const mg_plan *plan, mg_plan_stats *out) {
  clear_error();
  if (plan == nullptr || out == nullptr) {
    set_error("plan or out is NULL");
    return MG_ERR_INVALID_ARG;
  }
  *out = plan_stats(reinterpret_cast<const Plan *>(plan));
  return MG_OK;
}

int mg_plan_destroy(mg_plan *plan) {
  clear_error();
  plan_destroy(reinterpret_cast<Plan *>(plan));
  return MG_OK;
}

int mg_gemm_batched_noalloc(int dtype, int64_t count, const mg_problem *probs, void *stream) {
  clear_error();
  int rc = validate_batch(dtype, count, probs);
  if (rc != MG_OK) return rc;
  if (count == 0) return MG_OK;
  return gemm_batched_noalloc(dtype, count, probs, static_cast<hipStream_t>(stream));
}

int mg_gemm_batched(int dtype, int algo, int64_t count, const mg_problem *probs, void *stream) {
  clear_error();
  if (algo != MG_NATIVE && algo != MG_SPLIT_I8 && algo != MG_SPLIT_BF16) {
    set_error("unknown algo %d", algo);
    return MG_ERR_INVALID_ARG;
  }
  if (algo != MG_NATIVE && dtype != MG_F64) {
    set_error("split algorithms take FP64 operands");
    return MG_ERR_UNSUPPORTED;
  }
  reap_deferred(false);
  int rc = validate_batch(dtype, count, probs);
  if (rc != MG_OK) return rc;
  if (count == 0) return MG_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (algo != MG_NATIVE)  // built per call (its workspace is per call too)
    return gemm_split_batched(algo, count, probs, s);
  int dev = 0;
  MG_HIP_TRY(hipGetDevice(&dev));
  const uint64_t h = hash_problems(dtype, count, probs);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
      if (it->device != dev || it->dtype != dtype || it->hash != h ||
          (int64_t)it->probs.size() != count ||
          std::memcmp(it->probs.data(), probs, (size_t)count * sizeof(mg_problem)) != 0)
        continue;
      g_cache.splice(g_cache.begin(), g_cache, it);  // most recently used
      rc = plan_launch(it->plan, s, true);
      if (rc == MG_OK) MG_HIP_TRY(hipEventRecord(it->last, s));
      ++g_cache_hits;
      return rc;
    }
    ++g_cache_misses;
  }
  CachedBatch e;
  e.device = dev;
  e.dtype = dtype;
  e.hash = h;
  e.probs.assign(probs, probs + count);
  rc = plan_create(dtype, count, probs, nullptr, &e.plan);
  if (rc != MG_OK) return rc;
  rc = plan_launch(e.plan, s, true);  // captures the graph, then replays it
  if (rc == MG_OK && (hipEventCreateWithFlags(&e.last, hipEventDisableTiming) != hipSuccess ||
                      hipEventRecord(e.last, s) != hipSuccess)) {
    set_error("could not record completion event");
    rc = MG_ERR_HIP;
  }
  if (rc != MG_OK) {  // wait for anything enqueued, then free
    (void)hipStreamSynchronize(s);
    if (e.last) (void)hipEventDestroy(e.last);
    plan_destroy(e.plan);
    return rc;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.push_front(std::move(e));
  while (g_cache.size() > kPlanCacheSize) {
    CachedBatch &old = g_cache.back();
    {
      std::lock_guard<std::mutex> lk2(g_deferred_mu);
      g_deferred.emplace_back(old.plan, old.last);
    }
    g_cache.pop_back();
  }
  return MG_OK;
}

int mg_gemm_batched_cache_stats(int64_t *hits, int64_t *misses) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (hits) *hits = g_cache_hits;
  if (misses) *misses = g_cache_misses;
  return MG_OK;
}

}  // extern "C"
