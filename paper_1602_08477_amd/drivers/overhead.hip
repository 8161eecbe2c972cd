// Library overhead and naive-mapping measurement (the MI355X counterpart of
// the paper's zero-overhead and swapped-mapping experiments, Section 4.2,
// Figs. 5 and 6).  Prints one JSON object.
//
//   1. The same tiled kernel reached two ways: through the C ABI (mg_gemm:
//      validation, work-division rule, dispatch) and by launching the kernel
//      template directly with hipLaunchKernelGGL.  Reported: device time per
//      launch (HIP events around back-to-back launches) and host time per
//      enqueue (wall time of batches of enqueues, the device drained between
//      batches).
//   2. The naive one-output-per-lane work division (MG_NAIVE_CFG) against the
//      library's pick, device time per launch.
//
// Usage: mg_overhead [reps]   (links libmg.so; inputs U[-1,1) from a fixed
// integer hash, the outputs are not checked here: the test suite does that)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <vector>

#include "../csrc/gemm_launch.h"

namespace {

#define CK(x)                                                                          \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      fprintf(stderr, "%s failed: %s (line %d)\n", #x, hipGetErrorString(e_), __LINE__); \
      exit(1);                                                                         \
    }                                                                                  \
  } while (0)
#define CKMG(x)                                                                  \
  do {                                                                           \
    int r_ = (x);                                                                \
    if (r_ != MG_OK) {                                                           \
      fprintf(stderr, "%s failed: %d %s (line %d)\n", #x, r_, mg_last_error(), __LINE__); \
      exit(1);                                                                   \
    }                                                                            \
  } while (0)

__global__ void fill_kernel(double *p, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
  }
}

struct Mats {
  int n;
  double *A, *B, *C;
};

Mats make(int n) {
  Mats m{n, nullptr, nullptr, nullptr};
  const size_t bytes = (size_t)n * n * sizeof(double);
  CK(hipMalloc(&m.A, bytes));
  CK(hipMalloc(&m.B, bytes));
  CK(hipMalloc(&m.C, bytes));
  double *ps[3] = {m.A, m.B, m.C};
  for (int i = 0; i < 3; ++i)
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, 0, ps[i], (int64_t)n * n,
                       (uint64_t)(i + 1) << 40);
  CK(hipDeviceSynchronize());
  return m;
}

void drop(Mats &m) {
  CK(hipFree(m.A));
  CK(hipFree(m.B));
  CK(hipFree(m.C));
}

template <typename F>
double device_ms_per_launch(F launch, int reps, hipStream_t s) {
  for (int i = 0; i < 3; ++i) launch();
  CK(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) launch();
  CK(hipEventRecord(e1, s));
  CK(hipEventSynchronize(e1));
  float ms = 0;
  CK(hipEventElapsedTime(&ms, e0, e1));
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return ms / reps;
}

// Host wall time per enqueue: batches of `batch` enqueues timed, the stream
// drained (untimed) between batches so the queue never fills.
template <typename F>
double host_us_per_enqueue(F launch, int batches, int batch, hipStream_t s) {
  for (int i = 0; i < 8; ++i) launch();
  CK(hipStreamSynchronize(s));
  double total = 0;
  for (int b = 0; b < batches; ++b) {
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < batch; ++i) launch();
    const auto t1 = std::chrono::steady_clock::now();
    total += std::chrono::duration<double, std::micro>(t1 - t0).count();
    CK(hipStreamSynchronize(s));
  }
  return total / ((double)batches * batch);
}

mg::GemmArgs<double> args(const Mats &m) {
  mg::GemmArgs<double> g;
  g.A = m.A;
  g.B = m.B;
  g.C = m.C;
  g.lda = g.ldb = g.ldc = m.n;
  g.m = g.n = g.k = m.n;
  g.alpha = 1.0;
  g.beta = 1.0;
  return g;
}

// The kernel template mg_gemm picks for these shapes, launched directly.
template <typename K>
void direct(K kern, dim3 grid, int threads, size_t lds, const mg::GemmArgs<double> &g, int tm,
            int tn, hipStream_t s) {
  hipLaunchKernelGGL(kern, grid, dim3(threads), lds, s, g, tm, tn);
}

void one_shape(int n, int reps, hipStream_t s, bool first) {
  Mats m = make(n);
  const mg::GemmArgs<double> g = args(m);
  const int cfg = mg_pick_tile_cfg(MG_F64, n, n, n);
  int bm = 0, bn = 0, bk = 0, threads = 0;
  CKMG(mg_tile_cfg_info(MG_F64, cfg, &bm, &bn, &bk, &threads));
  const int tm = (n + bm - 1) / bm, tn = (n + bn - 1) / bn;
  auto lib_call = [&] {
    CKMG(mg_gemm(MG_F64, MG_NATIVE, n, n, n, 1.0, m.A, n, m.B, n, 1.0, m.C, n, s));
  };
  // direct launch of the same template instance
  std::function<void()> raw;
  if (cfg == 4) {
    typedef mg::TileShape<double, 32, 32, 2, 2, 1> S;
    raw = [&, tm, tn] {
      direct(mg::gemm_native_kernel<double, 32, 32, true, 2, 2, 1, false, false>,
             dim3(tm * tn), S::THREADS, S::LDS_BYTES, g, tm, tn, s);
    };
  } else if (cfg == 19 || cfg == 23 || cfg == 21 || cfg == 26) {
    if (cfg == 26) {
      typedef mg::DmaShape<double, 64, 64, 2, 2, 2, 2> S;
      auto k = mg::gemm_dma_kernel<double, 64, 64, 2, 2, 2, false, false, 2>;
      CK(hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS_BYTES));
      raw = [&, tm, tn, k] { direct(k, dim3(tm * tn), S::THREADS, S::LDS_BYTES, g, tm, tn, s); };
    } else if (cfg == 19) {
      typedef mg::DmaShape<double, 32, 32, 2, 2, 4> S;
      auto k = mg::gemm_dma_kernel<double, 32, 32, 2, 2, 4, false, false>;
      CK(hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS_BYTES));
      raw = [&, tm, tn, k] { direct(k, dim3(tm * tn), S::THREADS, S::LDS_BYTES, g, tm, tn, s); };
    } else if (cfg == 23) {
      typedef mg::DmaShape<double, 64, 64, 2, 2, 2> S;
      auto k = mg::gemm_dma_kernel<double, 64, 64, 2, 2, 2, false, false>;
      CK(hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS_BYTES));
      raw = [&, tm, tn, k] { direct(k, dim3(tm * tn), S::THREADS, S::LDS_BYTES, g, tm, tn, s); };
    } else {
      typedef mg::DmaShape<double, 128, 128, 2, 4, 2> S;
      auto k = mg::gemm_dma_kernel<double, 128, 128, 2, 4, 2, false, false>;
      CK(hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::LDS_BYTES));
      raw = [&, tm, tn, k] { direct(k, dim3(tm * tn), S::THREADS, S::LDS_BYTES, g, tm, tn, s); };
    }
  } else {
    fprintf(stderr, "no direct launcher for cfg %d\n", cfg);
    exit(1);
  }
  auto naive = [&] {
    CKMG(mg_gemm_cfg(MG_F64, MG_NAIVE_CFG, n, n, n, 1.0, m.A, n, m.B, n, 1.0, m.C, n, s));
  };
  // the two ways alternate in rounds (clock and thermal drift hit both
  // alike); the median round of each is reported
  const int r = n >= 4096 ? std::max(3, reps / 20) : reps;
  std::vector<double> t_lib, t_raw;
  for (int round = 0; round < 7; ++round) {
    t_lib.push_back(device_ms_per_launch(lib_call, r, s));
    t_raw.push_back(device_ms_per_launch(raw, r, s));
  }
  std::sort(t_lib.begin(), t_lib.end());
  std::sort(t_raw.begin(), t_raw.end());
  const double d_lib = t_lib[t_lib.size() / 2], d_raw = t_raw[t_raw.size() / 2];
  const double d_naive = device_ms_per_launch(naive, std::max(2, r / 10), s);
  double h_lib = -1, h_raw = -1;
  if (n <= 256) {
    h_lib = host_us_per_enqueue(lib_call, 40, 256, s);
    h_raw = host_us_per_enqueue(raw, 40, 256, s);
  }
  const double flop = 2.0 * n * (double)n * n;
  printf("%s{\"n\": %d, \"cfg\": %d, \"device_ms_mg_gemm\": %.6f, \"device_ms_direct\": %.6f, "
         "\"overhead_pct\": %.2f, \"device_ms_spread_mg_gemm\": [%.6f, %.6f], "
         "\"device_ms_spread_direct\": [%.6f, %.6f], "
         "\"tiled_tflops\": %.3f, \"naive_ms\": %.6f, \"naive_tflops\": %.3f, "
         "\"host_us_per_enqueue_mg_gemm\": %.3f, \"host_us_per_enqueue_direct\": %.3f}",
         first ? "" : ", ", n, cfg, d_lib, d_raw, 100.0 * (d_lib - d_raw) / d_raw, t_lib.front(),
         t_lib.back(), t_raw.front(), t_raw.back(), flop / d_raw / 1e9, d_naive,
         flop / d_naive / 1e9, h_lib, h_raw);
  fflush(stdout);
  drop(m);
}

}  // namespace

int main(int argc, char **argv) {
  const int reps = argc > 1 ? atoi(argv[1]) : 200;
  hipStream_t s;
  CK(hipStreamCreate(&s));
  printf("{\"shapes\": [");
  const int ns[] = {64, 256, 1024, 2048, 4096};
  for (int i = 0; i < 5; ++i) one_shape(ns[i], reps, s, i == 0);
  printf("]}\n");
  CK(hipStreamDestroy(s));
  return 0;
}
