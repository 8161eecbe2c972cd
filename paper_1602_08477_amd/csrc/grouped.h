// Batched (grouped) GEMM: plans, persistent kernel, graph replay, tuning.
#pragma once

#include <vector>

#include "common.h"
#include "gemm_native.h"

namespace mg {

constexpr int kNumGroupedClasses = MG_NUM_GROUPED_CLASSES;
constexpr int kTuneEdges = MG_TUNE_EDGES;

struct Plan;

// Bucket of a problem shape in the tuning table: per extent, bucket 0 holds
// [1, 32), bucket b in 1..4 holds [16*2^b, 32*2^b), bucket 5 holds [512, inf).
int tune_bucket(int64_t m, int64_t n, int64_t k);
int64_t tune_bucket_rep(int b);
int grouped_class_tile(int cls, int *bm, int *bn);
int heuristic_class(int64_t m, int64_t n);

// Host work list of a batch: tile records (device layout, problem arguments
// inline) sorted longest first, ready to be copied to the device as bytes.
struct WorkList {
  int dtype = MG_F64;
  int ntiles = 0;
  std::vector<unsigned char> tiles;
  mg_plan_stats stats{};
};

int build_worklist(int dtype, int64_t count, const mg_problem *probs, const mg_tune_table *table,
                   WorkList *out);
// Persistent grid (CUs x occupancy, at most ntiles) for the grouped kernel.
int grouped_grid(int dtype, int ntiles, int *grid, int *occupancy);
// Enqueues the persistent kernel over a device copy of a work list.
int launch_worklist(int dtype, const void *d_tiles, int ntiles, int grid, hipStream_t s);

int plan_create(int dtype, int64_t count, const mg_problem *probs, const mg_tune_table *table,
                Plan **out);
int plan_launch(Plan *p, hipStream_t s, bool use_graph);
void plan_destroy(Plan *p);
const mg_plan_stats &plan_stats(const Plan *p);

// Largest work list (bytes) of gemm_batched_noalloc: 8 MiB, about 87 000
// FP64 tiles (96 bytes each).
constexpr size_t kNoAllocWorklistBytes = (size_t)8 << 20;
// One-shot batch whose work list goes to a static per-device buffer.
int gemm_batched_noalloc(int dtype, int64_t count, const mg_problem *probs, hipStream_t s);

// Times every tile class on every shape bucket and records the fastest.
int autotune(int dtype, int reps, hipStream_t s, mg_tune_table *out);
// autotune through the JSON cache at `path` (NULL or "": no cache).
int autotune_cached(int dtype, int reps, const char *path, hipStream_t s, mg_tune_table *out,
                    int *from_cache);

}  // namespace mg
