// Drives the C ABI's host-side paths (argument validation, layout queries,
// work-division rules, tuning-table helpers, batch validation, the server's
// request validation in host-simulation mode) under AddressSanitizer and
// UndefinedBehaviorSanitizer.  No call here reaches a GPU: every matrix
// pointer is a fake, aligned address that validation inspects but nothing
// dereferences, and every call is one that must fail before enqueueing or
// return early (m == 0).
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mg.h"

static int failures = 0;

#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      std::fprintf(stderr, "line %d: expected %s (last error: %s)\n", __LINE__,   \
                   #cond, mg_last_error());                                       \
      ++failures;                                                                 \
    }                                                                             \
  } while (0)

static void *fake(uint64_t i) { return reinterpret_cast<void *>(0x100000000ull + (i << 28)); }

int main() {
  void *A = fake(1), *B = fake(2), *C = fake(3);
  // plain GEMM: every argument error, then the m == 0 no-op
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, -1, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(std::strlen(mg_last_error()) > 0);
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, 4, 4, 4, 1, A, 3, B, 4, 0, C, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, 4, 4, 4, 1, nullptr, 4, B, 4, 0, C, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, 4, 4, 4, 1, A, 4, B, 4, 0, A, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm(MG_F64, 7, 4, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) != MG_OK);
  EXPECT(mg_gemm(MG_F32, MG_SPLIT_I8, 4, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) != MG_OK);
  EXPECT(mg_gemm(5, MG_NATIVE, 4, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) != MG_OK);
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, 0, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) == MG_OK);
  EXPECT(mg_gemm(MG_F64, MG_NATIVE, INT64_MAX / 2, INT64_MAX / 2, 4, 1, A, 4, B, INT64_MAX / 2,
                 0, C, INT64_MAX / 2, nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_cfg(MG_F64, 999, 4, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_ex(MG_F64, -1, 2, 0, 4, 4, 4, 1, A, 4, B, 4, 0, C, 4, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_ex(MG_F64, -1, 1, 0, 4, 8, 4, 1, A, 3, B, 8, 0, C, 8, nullptr) ==
         MG_ERR_INVALID_ARG);
  // DAXPY
  EXPECT(mg_daxpy(-1, 1.0, (double *)A, 1, (double *)B, 1, nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_daxpy(8, 1.0, (double *)A, 0, (double *)B, 1, nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_daxpy(8, 1.0, (double *)A, 1, (double *)A + 3, 1, nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_daxpy(8, 1.0, (double *)((char *)A + 4), 1, (double *)B, 1, nullptr) ==
         MG_ERR_INVALID_ARG);
  EXPECT(mg_daxpy(0, 1.0, (double *)A, 1, (double *)B, 1, nullptr) == MG_OK);
  // work divisions
  const int ncfg = mg_num_tile_cfgs();
  EXPECT(ncfg > 0);
  for (int c = 0; c < ncfg; ++c) {
    int bm = 0, bn = 0, bk = 0, th = 0;
    EXPECT(mg_tile_cfg_info(MG_F64, c, &bm, &bn, &bk, &th) == MG_OK);
    EXPECT(bm > 0 && bn > 0 && bk > 0 && th > 0);
    EXPECT(mg_tile_cfg_info(MG_F32, c, nullptr, nullptr, nullptr, nullptr) == MG_OK);
  }
  EXPECT(mg_tile_cfg_info(MG_F64, ncfg, nullptr, nullptr, nullptr, nullptr) ==
         MG_ERR_INVALID_ARG);
  for (int64_t s : {1, 17, 512, 1024, 1536, 2048, 4096, 8192}) {
    const int c = mg_pick_tile_cfg(MG_F64, s, s, s);
    EXPECT(c >= 0 && c < ncfg);
    EXPECT(mg_pick_tile_cfg(MG_F32, s, s, s) >= 0);
  }
  // split workspace layout
  for (int algo : {MG_SPLIT_I8, MG_SPLIT_BF16}) {
    EXPECT(mg_split_default_slices(algo) > 0);
    for (int64_t s : {0, 1, 255, 257, 4096}) {
      mg_split_layout L;
      std::memset(&L, 0xff, sizeof L);
      EXPECT(mg_split_layout_query(algo, 7, s, s + 1, s + 2, &L) == MG_OK);
      EXPECT(L.e_off % 256 == 0 && L.f_off % 256 == 0 && L.a_off % 256 == 0 &&
             L.b_off % 256 == 0 && L.total_bytes >= L.b_off);
    }
    mg_split_layout L;
    EXPECT(mg_split_layout_query(algo, 0, 4, 4, 4, &L) == MG_ERR_INVALID_ARG);
    EXPECT(mg_split_layout_query(algo, 17, 4, 4, 4, &L) == MG_ERR_INVALID_ARG);
    EXPECT(mg_split_layout_query(algo, 7, -4, 4, 4, &L) == MG_ERR_INVALID_ARG);
  }
  EXPECT(mg_split_default_slices(MG_NATIVE) < 0 || mg_split_default_slices(MG_NATIVE) == 0 ||
         true);
  EXPECT(mg_split_prepare(MG_SPLIT_I8, 7, 64, 64, 64, (double *)A, 64, (double *)B, 64, C, 16,
                          nullptr) == MG_ERR_INVALID_ARG);  // workspace too small
  // tuning-table helpers
  for (int c = 0; c < MG_NUM_GROUPED_CLASSES; ++c) {
    int bm = 0, bn = 0;
    EXPECT(mg_grouped_class_info(c, &bm, &bn) == MG_OK && bm > 0 && bn > 0);
  }
  EXPECT(mg_grouped_class_info(MG_NUM_GROUPED_CLASSES, nullptr, nullptr) != MG_OK);
  for (int64_t x : {1, 16, 31, 32, 63, 64, 511, 512, 100000}) {
    const int b = mg_tune_bucket(x, x, x);
    EXPECT(b >= 0 && b < MG_TUNE_BUCKETS);
  }
  mg_tune_table t;
  EXPECT(mg_tune_default(MG_F64, &t) == MG_OK);
  for (int i = 0; i < MG_TUNE_BUCKETS; ++i)
    EXPECT(t.cls[i] >= 0 && t.cls[i] < MG_NUM_GROUPED_CLASSES);
  // batches: an invalid problem is named by index; overlapping outputs rejected
  std::vector<mg_problem> probs(5);
  for (int i = 0; i < 5; ++i)
    probs[i] = mg_problem{8, 8, 8, 1.0, 1.0, fake(10 + 3 * i), 8, fake(11 + 3 * i), 8,
                          fake(12 + 3 * i), 8};
  probs[3].lda = 2;
  EXPECT(mg_gemm_batched(MG_F64, MG_NATIVE, 5, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(std::strstr(mg_last_error(), "3") != nullptr);
  EXPECT(mg_gemm_batched_noalloc(MG_F64, 5, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  mg_plan *plan = nullptr;
  EXPECT(mg_plan_create(MG_F64, 5, probs.data(), nullptr, &plan) == MG_ERR_INVALID_ARG);
  probs[3].lda = 8;
  probs[4].C = probs[2].C;
  EXPECT(mg_gemm_batched(MG_F64, MG_NATIVE, 5, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_batched(MG_F64, MG_NATIVE, -1, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_batched(MG_F64, MG_NATIVE, 0, nullptr, nullptr) == MG_OK);
  EXPECT(mg_gemm_batched(MG_F32, MG_SPLIT_I8, 5, probs.data(), nullptr) == MG_ERR_UNSUPPORTED);
  EXPECT(mg_gemm_batched(MG_F64, 9, 5, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_batched(MG_F64, MG_SPLIT_BF16, 5, probs.data(), nullptr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_gemm_batched(MG_F64, MG_SPLIT_I8, 0, nullptr, nullptr) == MG_OK);
  EXPECT(mg_gemm_batched_noalloc(MG_F64, 0, nullptr, nullptr) == MG_OK);
  // server request validation (host simulation: nothing touches a device)
  mg_server_opts o{};
  o.n_streams = 2;
  o.max_slots = 4;
  o.max_queue = 8;
  o.max_batch = 4;
  o.hbm_budget_bytes = 1 << 20;
  o.simulate = 1;
  o.sim_tflops = 1.0;
  mg_server *srv = nullptr;
  mg_server_opts bad = o;
  bad.n_streams = 0;
  EXPECT(mg_server_create(&bad, &srv) == MG_ERR_INVALID_ARG && srv == nullptr);
  EXPECT(mg_server_create(&o, &srv) == MG_OK && srv != nullptr);
  mg_request r{};
  r.dtype = MG_F64;
  r.algo = MG_NATIVE;
  r.p = mg_problem{64, 64, 64, 1.0, 1.0, A, 64, B, 64, C, 64};
  uint64_t ticket = 0;
  mg_request big = r;
  big.p = mg_problem{512, 512, 512, 1.0, 1.0, A, 512, B, 512, C, 512};
  EXPECT(mg_gemm_submit(srv, &big, &ticket) == MG_ERR_NO_MEMORY);
  mg_request ov = r;
  ov.p.C = A;
  EXPECT(mg_gemm_submit(srv, &ov, &ticket) == MG_ERR_INVALID_ARG);
  mg_request f32split = r;
  f32split.dtype = MG_F32;
  f32split.algo = MG_SPLIT_I8;
  EXPECT(mg_gemm_submit(srv, &f32split, &ticket) == MG_ERR_UNSUPPORTED);
  EXPECT(mg_gemm_submit(srv, &r, &ticket) == MG_OK);
  mg_result res{};
  EXPECT(mg_gemm_wait(srv, ticket, &res) == MG_OK && res.status == MG_OK);
  EXPECT(mg_gemm_poll(srv, ticket, &res) == MG_ERR_NOT_FOUND);
  EXPECT(mg_gemm_submit(nullptr, &r, &ticket) == MG_ERR_INVALID_ARG);
  mg_server_stats st{};
  EXPECT(mg_server_get_stats(srv, &st) == MG_OK && st.completed == 1 && st.rejected_memory == 1);
  mg_request rev[2] = {r, r};
  rev[0].t_arrival_ns = 10;
  rev[1].t_arrival_ns = 5;
  mg_result rr[2];
  EXPECT(mg_server_replay(srv, 2, rev, rr) == MG_ERR_INVALID_ARG);
  EXPECT(mg_server_destroy(srv) == MG_OK);
  std::printf("C ABI under sanitizers: %d failures\n", failures);
  return failures != 0;
}
