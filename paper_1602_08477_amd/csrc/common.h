// Internal helpers shared by the HIP translation units of libmg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mg.h"

namespace mg {

// ------------------------------------------------------------ error state
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define MG_HIP_TRY(expr)                                                        \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::mg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                      __FILE__, __LINE__);                                      \
      return MG_ERR_HIP;                                                        \
    }                                                                           \
  } while (0)

// ------------------------------------------------------------- vector types
typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// ------------------------------------------------- LDS poison (debug) --
// Built with -DMG_LDS_POISON (the debug library variant), every LDS stage is
// filled with 0xFF bytes (NaN as FP64 / FP32 / BF16, -1 as INT8) before it is
// (re)filled, then the LDS writes are waited for and the workgroup
// synchronises (no wait on vector memory, so loads in flight stay in flight).
// A read of a stage before its data has landed, or of bytes no load writes,
// then changes the result; the normal build compiles this to nothing.
#ifdef MG_LDS_POISON
__device__ __forceinline__ void lds_poison(void *p, int bytes) {
  typedef __attribute__((address_space(3))) int lds_int;
  lds_int *q = (lds_int *)(__attribute__((address_space(3))) void *)p;
  for (int o = (int)threadIdx.x; o < bytes / 4; o += (int)blockDim.x) q[o] = -1;
  // lgkmcnt(0); vmcnt and expcnt at their maxima (not waited for)
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
}
#define MG_LDS_POISON_STAGE(p, bytes) ::mg::lds_poison((p), (bytes))
#else
#define MG_LDS_POISON_STAGE(p, bytes) ((void)0)
#endif

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Number of XCDs workgroups are dealt round-robin over on MI355X.
constexpr int kNumXcd = 8;

// Tile id for workgroup `b` of `T`: consecutive tile ids land on the same
// XCD (and so share its L2).  The dispatcher deals workgroups to XCDs in
// turn, so XCD x runs workgroups x, x+8, x+16, ...; give it a contiguous
// block of tile ids instead.
__device__ __forceinline__ int xcd_remap(int b, int T) {
  const int x = b % kNumXcd, loc = b / kNumXcd;
  const int per = T / kNumXcd, rem = T % kNumXcd;
  const int start = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  return start + loc;
}

// Grouped raster: tile t -> (tm, tn) walking `group` tile-rows at a time so
// that concurrently running tiles share A row panels and B column panels.
__device__ __forceinline__ void grouped_tile(int t, int tiles_m, int tiles_n, int group,
                                             int &tm, int &tn) {
  const int per_group = group * tiles_n;
  const int g = t / per_group;
  const int first = g * group;
  const int gsize = min(group, tiles_m - first);
  const int r = t - g * per_group;
  tm = first + r % gsize;
  tn = r / gsize;
}

// Byte range [lo, hi) touched by a rows x cols row-major matrix of pitch ld.
inline void byte_span(const void *p, int64_t rows, int64_t cols, int64_t ld, int64_t esz,
                      uintptr_t &lo, uintptr_t &hi) {
  lo = reinterpret_cast<uintptr_t>(p);
  hi = lo + (uintptr_t)(((rows - 1) * ld + cols) * esz);
}

inline bool spans_overlap(const void *a, int64_t ar, int64_t ac, int64_t ald, const void *b,
                          int64_t br, int64_t bc, int64_t bld, int64_t esz) {
  if (ar <= 0 || ac <= 0 || br <= 0 || bc <= 0) return false;
  uintptr_t a0, a1, b0, b1;
  byte_span(a, ar, ac, ald, esz, a0, a1);
  byte_span(b, br, bc, bld, esz, b0, b1);
  return a0 < b1 && b0 < a1;
}

// Validates one GEMM problem; sets the error message and returns an MG_ERR
// code, or MG_OK.  `what` prefixes the message (e.g. "problem 12").
int validate_problem(const char *what, int64_t m, int64_t n, int64_t k, double alpha,
                     const void *A, int64_t lda, const void *B, int64_t ldb, double beta,
                     const void *C, int64_t ldc, int64_t esz);

// Same for C <- alpha*op(A)*op(B) + beta*C: A stored k x m when ta, B stored
// n x k when tb.
int validate_problem_op(const char *what, bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                        double alpha, const void *A, int64_t lda, const void *B, int64_t ldb,
                        double beta, const void *C, int64_t ldc, int64_t esz);

}  // namespace mg
