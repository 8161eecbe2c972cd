// Split-precision FP64 GEMM: FP64 operands are cut into exact integer slices
// with per-row (A) and per-column (B) power-of-two scales, the slice products
// run on INT8 (INT32 accumulation) or BF16 (FP32 accumulation) matrix cores,
// and FP64 is used only for scaling, slicing and the final recombination.
#pragma once

#include "common.h"

namespace mg {

// Padding granularity of the workspace copies: rows of A and columns of B
// (the largest product tile), and k (one LDS stage).
constexpr int kSplitTileMN = 256;
constexpr int kSplitTileK = 128;
constexpr int kSplitMaxSlices = 16;

struct SplitLayout {
  int64_t mp, np, kp;    // padded extents
  int64_t elem_bytes;    // 1 (INT8 slices) or 2 (BF16 slices)
  int64_t e_off, f_off;  // int32 exponents of A rows [mp], B columns [np]
  int64_t a_off, b_off;  // A slices [s][mp][kp], B slices [s][np][kp] (B transposed)
  int64_t p_off;         // FP64 partial sums of the recombination [mp][np]
  int64_t total;         // bytes
};

int split_default_slices(int algo);
int split_bits(int algo);
int split_layout(int algo, int slices, int64_t m, int64_t n, int64_t k, SplitLayout *L);

// Scales + slices of A and B into the workspace (validated arguments).
int split_prepare(int algo, int slices, int64_t m, int64_t n, int64_t k, const double *A,
                  int64_t lda, const double *B, int64_t ldb, void *ws, hipStream_t s);

// Work divisions of the product kernel; cfg < 0 picks by size.
int split_num_cfgs();
// `latency`: one call on an otherwise idle device (the all-pairs 64x64 tile at
// the default slice count up to n = 2048 INT8 / 1024 BF16, the pair-parallel
// division for other slice counts below one 128x128 tile per CU); false: a
// device shared with other work
// (fused divisions only, the most throughput per FLOP).  Both give the same
// bits.
int split_pick_cfg(int algo, int slices, int64_t mp, int64_t np, bool latency);
// Workspace bytes the division `cfg` needs (<= the layout's total), and
// those of the division split_pick_cfg would pick.
int64_t split_ws_needed(const SplitLayout &L, int cfg);
int64_t split_workspace_bytes(int algo, int slices, int64_t m, int64_t n, int64_t k,
                              bool latency);

// Slice products + recombination + epilogue from a prepared workspace.
int split_multiply(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                   double beta, double *C, int64_t ldc, void *ws, hipStream_t s, int cfg = -1);

// prepare + multiply with a caller-provided workspace.
int gemm_split(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
               double *C, int64_t ldc, void *ws, int64_t ws_bytes, hipStream_t s, int cfg = -1);

// The same with a workspace from the library's stream-ordered pool on `s`, of
// the size the picked division needs (see split_pick_cfg for `latency`).
int gemm_split_pooled(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                      double *C, int64_t ldc, hipStream_t s, bool latency = true);

// The library's stream-ordered pool for split workspaces on the current
// device (freed blocks are kept for reuse), and a trim of every such pool.
int workspace_pool(hipMemPool_t *out);
int release_workspace_pools();

// Device workspace and pinned host staging that a caller who runs batches one
// after another on one stream keeps between calls (the server's lanes), so a
// batch allocates and frees nothing; grown on demand, never shrunk.
struct SplitBatchBuffers {
  void *d = nullptr, *h = nullptr;
  size_t d_cap = 0, h_cap = 0;
  // Grows the buffers (hipMalloc / hipHostMalloc); the caller guarantees that
  // no work still uses them.
  int reserve(size_t dev_bytes, size_t host_bytes);
  void release();
};

// Many independent FP64 problems (validated descriptors) in one set of
// launches, at the default slice count: per-problem workspaces in one
// allocation (from the workspace pool, freed on `s` after the batch; or in
// `buf`, whose previous contents must no longer be in use), batched
// preparation, one product launch over the 64x64 output tiles of all
// problems.  Each result equals a single call's bit for bit.
int gemm_split_batched(int algo, int64_t count, const mg_problem *probs, hipStream_t s,
                       SplitBatchBuffers *buf = nullptr);

}  // namespace mg
