/*
 * mg.h -- C ABI of the MI355X (gfx950) GEMM library.
 *
 * The operation is the generalised matrix-matrix multiply of the Alpaka
 * paper's evaluation (Section 4.2, "Performance"):
 *
 *     C <- alpha * A * B + beta * C,   A: m x k, B: k x n, C: m x n.
 *
 * Conventions shared by every entry point
 *  - Matrices are row-major 1-D buffers with a row pitch ("leading dimension",
 *    ld) in elements, ld >= number of columns: the paper's memory model of a
 *    plain pointer plus extent plus pitch (Section 3.4, "Memory").
 *  - All matrix pointers are DEVICE pointers owned by the caller.  The library
 *    never allocates, frees, copies or migrates them (no implicit data
 *    movement, Section 3.1).  Host arrays of descriptors are read during the
 *    call only.
 *  - `stream` is a hipStream_t passed as void*; work is enqueued on it in
 *    order and the call returns without waiting (an asynchronous stream in the
 *    paper's sense, Section 3.4, "Streams").  There is no default stream or
 *    current-device assumption beyond HIP's own: the stream must belong to the
 *    calling thread's current device.
 *  - Return value: MG_OK (0) or a negative MG_ERR_* code.  Argument errors are
 *    detected before anything is enqueued.  mg_last_error() returns a
 *    thread-local message describing the most recent failure of the calling
 *    thread.
 *  - BLAS special cases: beta == 0 means C is not read (NaN in C does not
 *    propagate); alpha == 0 or k == 0 means A and B are not read and
 *    C <- beta*C; m == 0 or n == 0 is a no-op.
 *  - The output C must not overlap A or B.
 */
#ifndef MG_H
#define MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define MG_OK 0
#define MG_PENDING 1            /* mg_gemm_poll: request not finished yet     */
#define MG_ERR_INVALID_ARG (-1) /* bad pointer/size/pitch/overlap/option      */
#define MG_ERR_UNSUPPORTED (-2) /* dtype x algo combination not provided      */
#define MG_ERR_HIP (-3)         /* HIP runtime error (message in last_error)  */
#define MG_ERR_NO_MEMORY (-4)   /* request larger than the HBM budget, or a
                                   device allocation failed                   */
#define MG_ERR_BUSY (-5)        /* server queue full                          */
#define MG_ERR_NOT_FOUND (-6)   /* unknown ticket                             */

/* ------------------------------------------------------------ element types */
#define MG_F64 0
#define MG_F32 1

/* -------------------------------------------------------------- algorithms */
#define MG_NATIVE 0     /* FP64 (or FP32) MFMA tiled kernel                   */
#define MG_SPLIT_I8 1   /* FP64 from INT8 slices, INT32 accumulation          */
#define MG_SPLIT_BF16 2 /* FP64 from BF16-held 8-bit slices, FP32 accumulation */

/* Message for the calling thread's most recent error ("" if none). The
 * pointer stays valid until the thread's next library call. */
const char *mg_last_error(void);

/* Library ABI version (major*10000 + minor*100 + patch). */
int mg_version(void);

/* Build variant: MG_BUILD_LDS_POISON is set in the debug build whose kernels
 * fill every LDS stage with 0xFF bytes before refilling it (race checks; the
 * release build returns 0). */
#define MG_BUILD_LDS_POISON 1
int mg_build_flags(void);

/* ------------------------------------------------------------ plain GEMM --
 * mg_gemm: C <- alpha*A*B + beta*C (Section 4.2 problem statement).
 *   dtype  MG_F64 (algo MG_NATIVE, MG_SPLIT_I8 or MG_SPLIT_BF16; the split
 *          algorithms take FP64 in and out) or MG_F32 (MG_NATIVE only).
 *   m,n,k  extents (>= 0).  lda >= k, ldb >= n, ldc >= n (elements).
 *   A,B,C  device pointers to dtype elements, naturally aligned.
 * The work division (macro-tile shape, i.e. blocks, threads per block and
 * elements per thread in the paper's terms, Table 2 and Section 3.4) is
 * chosen by the library from the shape.  The split algorithms use the
 * default slice count (mg_split_default_slices) and take their workspace
 * from the library's stream-ordered workspace pool on `stream` (released on
 * the same stream; see mg_release_cached_memory); use mg_gemm_split to
 * supply the workspace instead. */
int mg_gemm(int dtype, int algo, int64_t m, int64_t n, int64_t k, double alpha,
            const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
            void *C, int64_t ldc, void *stream);

/* Work divisions of the native kernel.  Configuration `cfg` in
 * [0, mg_num_tile_cfgs()) is a macro-tile of bm x bn outputs per workgroup
 * with a k-step of bk, computed by `threads` lanes.  MG_NAIVE_CFG (25) is
 * the naive mapping of the paper's portability experiment
 * (Section 4.2, Fig. 6): one output per lane, a 16 x 16 workgroup, no shared
 * memory, the k loop reading global memory (bm = bn = 16, bk = 1, threads =
 * 256; at most 65535 * 16 rows).  Returns MG_OK or MG_ERR_INVALID_ARG for an
 * unknown cfg; any output pointer may be NULL. */
#define MG_NAIVE_CFG 25
int mg_num_tile_cfgs(void);
int mg_tile_cfg_info(int dtype, int cfg, int *bm, int *bn, int *bk, int *threads);

/* mg_gemm with an explicit work division `cfg` (MG_NATIVE only).  Same
 * arguments and errors as mg_gemm; MG_ERR_INVALID_ARG for an unknown cfg. */
int mg_gemm_cfg(int dtype, int cfg, int64_t m, int64_t n, int64_t k, double alpha,
                const void *A, int64_t lda, const void *B, int64_t ldb,
                double beta, void *C, int64_t ldc, void *stream);

/* The cfg mg_gemm picks for this shape (its work-division rule). */
int mg_pick_tile_cfg(int dtype, int64_t m, int64_t n, int64_t k);

/* mg_gemm_ex: C <- alpha*op(A)*op(B) + beta*C on the native kernels, with
 * op(X) = X (trans 0) or its transpose X^T (trans 1).  The paper measures
 * square row-major operands only (Section 4.2); the transposed layouts run
 * the same tiles with the stored rows of A^T / B^T staged as k rows / k
 * columns, so every output sums the same products in the same order as the
 * plain layout (bit-identical results for the same cfg).
 *   transa 0: A stored m x k, lda >= k;  1: A stored k x m, lda >= m.
 *   transb 0: B stored k x n, ldb >= n;  1: B stored n x k, ldb >= k.
 *   cfg    a work division as in mg_gemm_cfg, or -1 for mg_pick_tile_cfg's.
 *   dtype  MG_F64 or MG_F32.  Other arguments, special cases and errors as
 *          mg_gemm (MG_ERR_INVALID_ARG for trans flags other than 0/1). */
int mg_gemm_ex(int dtype, int cfg, int transa, int transb, int64_t m, int64_t n, int64_t k,
               double alpha, const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
               void *C, int64_t ldc, void *stream);

/* ----------------------------------------------------------------- DAXPY --
 * mg_daxpy: y <- alpha*x + y (the vector operation of the paper's conceptual
 * comparison, Section 4.1).  Element i of x is x[i*incx], of y y[i*incy].
 *   n          number of elements (>= 0).
 *   incx, incy increments in elements, >= 1 (no reverse traversal).
 *   x, y       DEVICE pointers to doubles (8-byte aligned), owned by the
 *              caller; y may be x itself when incx == incy, no other overlap.
 * Each element is one fused multiply-add: y[i] = alpha*x[i] + y[i] rounded
 * once to the nearest double (ties to even), bit-identical for every launch
 * shape.  BLAS quick return: n == 0 or alpha == 0 leaves y untouched and reads
 * nothing (NaN in x does not propagate).  Asynchronous on `stream`.
 * Returns MG_OK or MG_ERR_INVALID_ARG (negative n, increment < 1, NULL or
 * misaligned pointer, overlap, extent overflow), MG_ERR_HIP on launch error. */
int mg_daxpy(int64_t n, double alpha, const double *x, int64_t incx, double *y, int64_t incy,
             void *stream);

/* ------------------------------------------------ split-precision FP64 --
 * The FP64 product is rebuilt from exact integer slices (not part of the
 * paper, which computes DGEMM natively; the splitting follows Ozaki et al.'s
 * error-free transformation of matrix products):
 *   1. E_i = frexp exponent of max_p |A[i][p]| (so |A[i][:]| < 2^E_i), F_j
 *      likewise for column j of B; an all-zero row/column gets 0.
 *   2. With r = x*2^-E and b = 7 (MG_SPLIT_I8) or 8 (MG_SPLIT_BF16), for
 *      t = 1..s: y = r*2^b, slice_t = trunc(y), r = y - slice_t (all exact,
 *      |slice_t| <= 2^b - 1).
 *   3. P_d = sum over p+q = d of A_p*B_q for d = 2..s+1, exactly (INT8 x INT8
 *      with INT32 accumulation, or BF16 x BF16 with FP32 accumulation over
 *      256-long k chunks, both exact for the integers involved).
 *   4. acc = sum_d P_d*2^(-b*d) in FP64, increasing d;
 *      C <- alpha*(2^(E_i+F_j)*acc) + beta*C, each product and the sum
 *      rounded once (no fused multiply-add).
 * Finite inputs are assumed.  Error vs the exact product is bounded per
 * element by |alpha| k 2^(E_i+F_j) (s+3) 2^(-b s) plus FP64 rounding.
 *
 * Workspace layout (bytes from the workspace base; all offsets 256-aligned):
 *   mp, np = m, n rounded up to 256; kp = k rounded up to 128 (all >= 1)
 *   int32 E[mp] at e_off, int32 F[np] at f_off (padding entries 0)
 *   A slices at a_off: [s][mp][kp] row-major elements (INT8, or BF16 bits)
 *   B slices at b_off: [s][np][kp], i.e. slice t of B transposed (k fastest)
 *   padding (rows >= m, columns >= n, k >= k) is zero.
 *   p_off: the product kernels' scratch up to total_bytes: FP64 partial sums
 *   [mp][np], or, for shapes the pair-parallel division serves, its INT32
 *   partial diagonal sums (larger; total_bytes accounts for it).
 */
typedef struct mg_split_layout {
  int64_t mp, np, kp, elem_bytes;
  int64_t e_off, f_off, a_off, b_off, p_off, total_bytes;
} mg_split_layout;

/* Default slice count: 7 for MG_SPLIT_I8, 6 for MG_SPLIT_BF16. */
int mg_split_default_slices(int algo);

/* Fills *out with the workspace layout; MG_ERR_INVALID_ARG for a bad algo,
 * slices outside [1, 16] or negative extents. */
int mg_split_layout_query(int algo, int slices, int64_t m, int64_t n, int64_t k,
                          mg_split_layout *out);

/* Steps 1-2: writes E, F and the slices of A and B into `workspace`
 * (device memory of at least total_bytes, owned by the caller). */
int mg_split_prepare(int algo, int slices, int64_t m, int64_t n, int64_t k, const double *A,
                     int64_t lda, const double *B, int64_t ldb, void *workspace,
                     int64_t workspace_bytes, void *stream);

/* Steps 1-4 with a caller-provided workspace: C <- alpha*A*B + beta*C. */
int mg_gemm_split(int algo, int slices, int64_t m, int64_t n, int64_t k, double alpha,
                  const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                  double *C, int64_t ldc, void *workspace, int64_t workspace_bytes,
                  void *stream);

/* Work divisions of the slice-product kernel (all give identical bits):
 * 0: 128x128 tile on 4 wavefronts, register-staged double buffer;
 * with a ring of direct-to-LDS stages: 1: 128x128 on 4 (ring of 4),
 * 2: 128x256 on 8 (ring of 3), 3: 256x128 on 4 (ring of 3), 4: 256x256 on
 * 16 (ring of 2), 5: 128x256 on 8 (ring of 2); with 64-byte k stages:
 * 6: 256x256 on 8 (ring of 4), 7: 256x256 on 16 (ring of 4), 8: 128x256 on 8
 * (ring of 6); 9-14 further tile and ring shapes; 15: pair-parallel, for
 * shapes with fewer than 256 tiles of 128x128 (mp/128 * np/128 < 256): the
 * slice pairs are cut into groups, each workgroup sums one group's pairs for
 * one 128x128 tile and writes exact INT32 partial diagonal sums, and a second
 * kernel adds them and folds them into FP64 as the other divisions do
 * (MG_ERR_INVALID_ARG on larger shapes); 16: all-pairs, default slice count
 * only (MG_ERR_INVALID_ARG otherwise): a 64x64 tile on 4 wavefronts holds
 * every slice of its rows of A and columns of B for one 64-byte k stage in
 * LDS and forms all slice pairs from it, one exact INT32 sum per diagonal and
 * the FP64 partial sums in registers, two workgroups per CU (needs no
 * partial-sum region: p_off bytes of workspace suffice).  mg_gemm_split and
 * mg_gemm pick by size (16 at the default slice count: INT8 at every size,
 * BF16 up to n = 1024); mg_gemm_split_cfg takes cfg explicitly (-1 = pick).
 * MG_ERR_INVALID_ARG for an unknown cfg. */
int mg_split_num_cfgs(void);
int mg_gemm_split_cfg(int algo, int slices, int cfg, int64_t m, int64_t n, int64_t k,
                      double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                      double beta, double *C, int64_t ldc, void *workspace,
                      int64_t workspace_bytes, void *stream);

/* Split workspaces come from a stream-ordered pool the library creates per
 * device (the caller's default pool is not touched).  The pool keeps freed
 * blocks for reuse, so repeated calls do not go back to the device
 * allocator; this trims every such pool, returning the blocks no pending
 * work uses.  MG_OK, or MG_ERR_HIP. */
int mg_release_cached_memory(void);

/* ------------------------------------------------------- batched GEMM --
 * Many independent problems C_i <- alpha_i A_i B_i + beta_i C_i (each the
 * Section 4.2 operation) in ONE persistent launch.  A plan validates the
 * problems, picks a tile class per problem (from a tuning table or a
 * heuristic), builds a device work list of macro-tiles sorted longest first
 * (each record carries its problem's arguments), and on first launch
 * captures the persistent kernel in a HIP graph that later launches replay.
 * The grid is (CUs x occupancy) workgroups G; the list is dealt in rounds
 * of G tiles whose direction alternates (workgroup b takes tile b of round
 * 0, G-1-b of round 1, ...).  Blocks are independent and never synchronise
 * (Section 3.2), and every tile sums its k-steps in the order of the
 * single-problem kernels with one k group of wavefronts, so a problem's
 * result is the same whatever else is in the batch, and bit for bit equal to
 * mg_gemm_cfg on it alone with any one-k-group work division (0-24).  That
 * is also mg_gemm's own result unless mg_pick_tile_cfg picks a two-k-group
 * division (26-29; FP64 and FP32 problems with roughly 2^20 <= m*n < 2^22,
 * e.g. n = 1024 and 1536): those add two half-sums per output at the end, so
 * there the batched and single results agree to the rounding bound
 * (k+2)u(|alpha||A||B| + |beta||C|) per element, not bit for bit.
 * Problems may share A and B; no C may overlap another problem's C, A or B
 * (checked on the byte spans [first element, last element], so interleaved
 * sub-blocks of one buffer are rejected).  dtype MG_F64 or MG_F32. */
typedef struct mg_problem {
  int64_t m, n, k;
  double alpha, beta;
  const void *A;
  int64_t lda;
  const void *B;
  int64_t ldb;
  void *C;
  int64_t ldc;
} mg_problem;

#define MG_NUM_GROUPED_CLASSES 3 /* tile classes: 64x64, 64x32, 32x32    */
#define MG_TUNE_EDGES 6          /* per-extent buckets, see mg_tune_bucket */
#define MG_TUNE_BUCKETS 216      /* MG_TUNE_EDGES^3                        */

/* Tile class per shape bucket.  Bucket of an extent x: 0 for x < 32, b for
 * 16*2^b <= x < 32*2^b (b = 1..4), 5 for x >= 512; the table index is
 * (bucket(m)*6 + bucket(n))*6 + bucket(k). */
typedef struct mg_tune_table {
  int32_t dtype;
  int32_t cls[MG_TUNE_BUCKETS];
} mg_tune_table;

typedef struct mg_plan_stats {
  int64_t problems, tiles, workgroups, occupancy;
  int64_t tiles_per_class[MG_NUM_GROUPED_CLASSES];
  int64_t scale_tiles; /* tiles of problems with alpha == 0 or k == 0        */
  double flops;        /* sum of 2mnk                                        */
  double bytes;        /* sum of compulsory operand bytes                    */
  int64_t graph;       /* 1 once the launch has been captured in a graph     */
} mg_plan_stats;

typedef struct mg_plan mg_plan;

/* Macro-tile of tile class `cls`. */
int mg_grouped_class_info(int cls, int *bm, int *bn);
/* Index of (m, n, k) in mg_tune_table.cls. */
int mg_tune_bucket(int64_t m, int64_t n, int64_t k);
/* Heuristic table (largest tile wasting at most a quarter of its area). */
int mg_tune_default(int dtype, mg_tune_table *out);
/* Autotuner: for every bucket, times each tile class on a batch of problems
 * of the bucket's representative shape, as many (48 to 4096) as it takes for
 * the largest class to give every workgroup slot of the persistent kernel
 * four tiles, so that classes compete on throughput in a full batch (reps
 * launches on `stream`, HIP events), and records the fastest.  Allocates and
 * frees its own scratch operands (about 0.4 GB for FP64); blocks until done.
 * The work division is picked per architecture by measurement, as the paper
 * picks it per architecture (Section 4.2.3).  If the environment variable
 * MG_AUTOTUNE_CACHE names a file, this is mg_autotune_cached with that path. */
int mg_autotune(int dtype, int reps, void *stream, mg_tune_table *out);

/* mg_autotune through a persistent cache: a JSON file holding one table per
 * (device architecture name, CU count, dtype, library version).  A table
 * stored for the current device and dtype is returned without timing
 * (*from_cache = 1); otherwise the buckets are timed and the file is
 * rewritten with this table added or replaced (other entries kept; written
 * to a temporary name and renamed).  cache_path NULL or "" means no cache.
 * from_cache may be NULL.  MG_ERR_INVALID_ARG if the file cannot be written. */
int mg_autotune_cached(int dtype, int reps, const char *cache_path, void *stream,
                       mg_tune_table *out, int *from_cache);

/* Builds a plan (host work list + device copy; blocks while uploading).
 * `table` may be NULL (heuristic).  *out must be released with
 * mg_plan_destroy.  Errors: MG_ERR_INVALID_ARG naming the first bad problem
 * index, MG_ERR_HIP on allocation/copy failure. */
int mg_plan_create(int dtype, int64_t count, const mg_problem *probs,
                   const mg_tune_table *table, mg_plan **out);
/* Enqueues the whole batch on `stream` by replaying the plan's graph
 * (captured on first use). */
int mg_plan_launch(mg_plan *plan, void *stream);
/* The same two kernels launched directly (no graph). */
int mg_plan_launch_direct(mg_plan *plan, void *stream);
int mg_plan_get_stats(const mg_plan *plan, mg_plan_stats *out);
/* Frees the plan.  The caller must make sure no launch of it is pending. */
int mg_plan_destroy(mg_plan *plan);

/* One-shot: plan (heuristic table) + launch on `stream`.
 * MG_NATIVE: the plan of each distinct problem set is kept (the last 8 sets
 * per process, matched on device, dtype and every descriptor byte for byte)
 * with its launch captured in a HIP graph: a call whose problem set repeats
 * replays that graph instead of building and uploading a new work list (the
 * list holds pointers, extents and scalars only, so each replay reads the
 * operands' current contents).  An evicted plan's device memory is released
 * by a later library call once its last launch has completed.
 * MG_SPLIT_I8 / MG_SPLIT_BF16 (dtype MG_F64; MG_ERR_UNSUPPORTED otherwise):
 * the split-precision method of mg_gemm on every problem, with the default
 * slice count, in four launches for the whole batch -- exponents and slices
 * of all problems (three preparation grids), then one grid of 64x64 output
 * tiles over all problems, longest k first, each tile staging every slice of
 * its rows of A and columns of B per k stage and forming all slice pairs
 * from them, with the diagonal sums and FP64 partial sums in registers
 * (Section 3.3: independent grids of one device run concurrently; here they
 * share one launch).  The per-problem workspaces (exponents and
 * slices padded to 64 rows / columns and 64 k, in one allocation from the
 * library's workspace pool, freed on `stream` after the batch) and the
 * descriptors are built per call; nothing is kept.  Each result equals
 * mg_gemm(MG_F64, algo, ...) on that problem alone, bit for bit.
 * MG_ERR_NO_MEMORY if the workspaces cannot be allocated. */
int mg_gemm_batched(int dtype, int algo, int64_t count, const mg_problem *probs, void *stream);
/* Calls of mg_gemm_batched so far that replayed a kept plan (hits) and that
 * built a new one (misses).  Either pointer may be NULL. */
int mg_gemm_batched_cache_stats(int64_t *hits, int64_t *misses);

/* mg_gemm_batched_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same problems, validation, tile classes (heuristic table) and
 * results as mg_gemm_batched(dtype, MG_NATIVE, ...), bit for bit, but the
 * work list goes to a static 8 MiB device array (one per GPU, held until the
 * process ends; about 87 000 FP64 tiles) instead of library-allocated memory:
 * the call makes no hipMalloc/hipFree and creates no event.  It copies the
 * work list from host memory into that array on `stream` and launches the
 * persistent kernel behind it.  Every call on a GPU shares that GPU's
 * array: calls on one stream are ordered, but calls that overlap on one GPU
 * (other streams, other threads, before an earlier launch has finished on
 * another stream) race on it.  MG_ERR_INVALID_ARG (nothing enqueued) for a
 * batch whose work list exceeds the array, with the size in the message. */
int mg_gemm_batched_noalloc(int dtype, int64_t count, const mg_problem *probs, void *stream);

/* ----------------------------------------------------------- serving --
 * A request loop with continuous batching.  Requests (each one GEMM of the
 * Section 4.2 form, operands already on the device) are submitted from any
 * thread; a scheduler thread admits them in FIFO order while the admitted-
 * but-unfinished requests stay within `max_slots` and their bytes (A + B + C,
 * plus the split workspace for split requests) within `hbm_budget_bytes`, and
 * launches everything admitted so far as one batch on the next free stream
 * (one persistent grouped launch for the native requests, one batched split
 * launch set per split algorithm, as in mg_gemm_batched; each stream keeps
 * its own grow-only device workspace and pinned staging buffer for these,
 * so a batch allocates only when it needs more than any batch before it on
 * that stream; they are freed by mg_server_destroy).
 * Batches on different streams run concurrently on the
 * device (the paper's scheduler may run grids from several streams in
 * parallel, Section 3.3); requests that arrive while batches run are admitted
 * as slots and bytes free up and go out with the next batch.  A request's
 * arithmetic depends only on its own shape (fixed tile class table), so its
 * result is the same alone or in any mix.
 * The caller keeps every operand alive and unmodified until the request is
 * reported done; the library never copies operands.
 * Timestamps are steady-clock nanoseconds (mg_now_ns). */
typedef struct mg_server mg_server;

typedef struct mg_server_opts {
  int n_streams;            /* concurrent batches (1..8)                     */
  int max_slots;            /* admitted, unfinished requests (>= 1)          */
  int max_queue;            /* waiting (not admitted) requests (>= 1)        */
  int max_batch;            /* requests per batch (>= 1)                     */
  int64_t hbm_budget_bytes; /* admission cap on admitted request bytes       */
  const mg_tune_table *table; /* tile classes for native requests (NULL:
                                 heuristic); copied at creation              */
  /* Host simulation (capacity planning and host-logic tests): when nonzero
   * no HIP call is made and operands are never touched; a batch "runs" for
   * sim_launch_ns + (its FLOPs) / (sim_tflops * 1e12) seconds of host time,
   * with FLOPs counted as 2mnk (native) or pairs*2mnk at 2x rate (split). */
  int32_t simulate;
  double sim_tflops;
  int64_t sim_launch_ns;
} mg_server_opts;

typedef struct mg_request {
  int32_t dtype;          /* MG_F64 or MG_F32                                 */
  int32_t algo;           /* MG_NATIVE, or MG_SPLIT_I8 / MG_SPLIT_BF16 (F64)  */
  mg_problem p;
  int64_t t_arrival_ns;   /* scheduled arrival: latencies are measured from it */
  /* Producer event (hipEvent_t as void*) or NULL.  The server's streams do
   * not synchronise with the caller's, so the request's kernels are ordered
   * after the caller's writes to A, B and C only through this event: the lane
   * waits on it (hipStreamWaitEvent) before it launches the batch holding the
   * request.  The caller records it after those writes and keeps it alive and
   * un-recorded until the request is reported done.  With NULL the caller must
   * have finished every write to A, B and C (e.g. synchronised the producing
   * stream) before the call to mg_gemm_submit. */
  void *ready_event;
} mg_request;

typedef struct mg_result {
  int32_t status;         /* MG_OK or the request's error code               */
  int32_t batch_size;     /* requests in the batch it ran in                  */
  int64_t batch_id;
  int64_t t_arrival_ns, t_submit_ns, t_admit_ns, t_launch_ns, t_done_ns;
} mg_result;

typedef struct mg_server_stats {
  int64_t submitted, completed, rejected_busy, rejected_memory, failed;
  int64_t batches, max_batch_seen, max_inflight_bytes, max_slots_used;
} mg_server_stats;

/* Steady-clock time in nanoseconds (the server's clock). */
int64_t mg_now_ns(void);

/* Creates streams, buffers and threads on the calling thread's current
 * device.  MG_ERR_INVALID_ARG for out-of-range options. */
int mg_server_create(const mg_server_opts *opts, mg_server **out);
/* Finishes every submitted request, then releases everything. */
int mg_server_destroy(mg_server *s);
/* Non-blocking.  Validates the request (as mg_gemm); MG_ERR_NO_MEMORY if it
 * alone exceeds the budget, MG_ERR_BUSY if the waiting queue is full;
 * otherwise queues it and returns its ticket.  t_arrival_ns of 0 means "now". */
int mg_gemm_submit(mg_server *s, const mg_request *req, uint64_t *ticket);
/* MG_PENDING while the request runs; once done copies its result, releases
 * the ticket and returns MG_OK (the request's own status is in out->status).
 * MG_ERR_NOT_FOUND for an unknown or already released ticket. */
int mg_gemm_poll(mg_server *s, uint64_t ticket, mg_result *out);
/* Blocking variant of mg_gemm_poll. */
int mg_gemm_wait(mg_server *s, uint64_t ticket, mg_result *out);
int mg_server_get_stats(const mg_server *s, mg_server_stats *out);

/* Open-loop load generator: submits reqs[i] at t0 + reqs[i].t_arrival_ns
 * (t0 = time of the call; arrival offsets ascending) from a dedicated thread,
 * then waits for all of them and fills results[i] (absolute timestamps).
 * A rejected submission is reported in results[i].status. */
int mg_server_replay(mg_server *s, int64_t count, const mg_request *reqs, mg_result *results);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
