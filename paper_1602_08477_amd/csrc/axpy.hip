// DAXPY, y <- alpha*x + y (the vector kernel of the paper's conceptual
// comparison, Section 4.1): every element is one fused multiply-add, so the
// result is alpha*x[i] + y[i] rounded once, whatever the launch shape.
//
// The operation moves 24 bytes per element for 2 FLOP, far below the FP64
// ridge point: it is bound by HBM bandwidth.  Layout on MI355X: each lane
// moves one 16-byte chunk (two doubles) of x and of y with nontemporal
// loads and stores (streamed data that is never reused: kept out of the
// caches' way), one wavefront per workgroup, one workgroup per 1 KB span.
// Measured at n = 2^27 against wider workgroups (128-1024 lanes) and more
// chunks per lane (2-8, loads issued ahead of the FMAs): this shape keeps the
// most requests in flight across the 256 CUs and is the fastest.  Operands
// whose addresses differ in 16-byte phase, or with non-unit increments, take
// an element-wise kernel (8-byte accesses, still coalesced for unit stride).
#include <algorithm>

#include "axpy.h"

namespace mg {

namespace {

constexpr int kAxpyThreads = 256;   // element-wise kernel
constexpr int kAxpyVecThreads = 64;  // vector kernel: one wavefront

// x and y 16-byte aligned after `head` (0 or 1) leading elements; pairs
// [0, np) go through the vector path, the head and an odd last element are
// done by lanes 0 and 1 of workgroup 0.
__global__ __launch_bounds__(kAxpyVecThreads) void axpy_vec_kernel(int64_t n, int head,
                                                                    double alpha, const double *x,
                                                                    double *y) {
  const d2v *xv = reinterpret_cast<const d2v *>(x + head);
  d2v *yv = reinterpret_cast<d2v *>(y + head);
  const int64_t np = (n - head) >> 1;
  // one pass for any n below 2^31 pairs; longer vectors loop over the grid
  for (int64_t i = (int64_t)blockIdx.x * kAxpyVecThreads + threadIdx.x; i < np;
       i += (int64_t)gridDim.x * kAxpyVecThreads) {
    const d2v a = __builtin_nontemporal_load(xv + i);
    const d2v b = __builtin_nontemporal_load(yv + i);
    d2v r;
    r[0] = fma(alpha, a[0], b[0]);
    r[1] = fma(alpha, a[1], b[1]);
    __builtin_nontemporal_store(r, yv + i);
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    int64_t j = -1;
    if (threadIdx.x == 0 && head) j = 0;
    if (threadIdx.x == 1 && ((n - head) & 1)) j = n - 1;
    if (j >= 0) y[j] = fma(alpha, x[j], y[j]);
  }
}

// Any positive increments: element i of x at x[i*incx], of y at y[i*incy].
__global__ __launch_bounds__(kAxpyThreads) void axpy_elem_kernel(int64_t n, double alpha,
                                                                  const double *x, int64_t incx,
                                                                  double *y, int64_t incy) {
  for (int64_t i = (int64_t)blockIdx.x * kAxpyThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kAxpyThreads) {
    double *p = y + i * incy;
    *p = fma(alpha, x[i * incx], *p);
  }
}

}  // namespace

int axpy_f64(int64_t n, double alpha, const double *x, int64_t incx, double *y, int64_t incy,
             hipStream_t s) {
  if (n == 0 || alpha == 0.0) return MG_OK;
  const uintptr_t px = reinterpret_cast<uintptr_t>(x), py = reinterpret_cast<uintptr_t>(y);
  if (incx == 1 && incy == 1 && (px & 15) == (py & 15)) {
    const int head = (px & 15) ? 1 : 0;
    const int64_t np = std::max<int64_t>((n - head) >> 1, 0);
    // the dispatch's work-item count is 32-bit: at most 2^25 one-wave workgroups
    const int64_t blocks = std::min<int64_t>(
        std::max<int64_t>((np + kAxpyVecThreads - 1) / kAxpyVecThreads, 1), (int64_t)1 << 25);
    hipLaunchKernelGGL(axpy_vec_kernel, dim3((unsigned)blocks), dim3(kAxpyVecThreads), 0, s, n,
                       head, alpha, x, y);
  } else {
    // enough workgroups to cover the chip several times, each lane striding
    const int64_t blocks = std::min<int64_t>((n + kAxpyThreads - 1) / kAxpyThreads, 8192);
    hipLaunchKernelGGL(axpy_elem_kernel, dim3((unsigned)blocks), dim3(kAxpyThreads), 0, s, n,
                       alpha, x, incx, y, incy);
  }
  MG_HIP_TRY(hipGetLastError());
  return MG_OK;
}

}  // namespace mg
