// Drives the serving loop's threads (scheduler, per-lane completion waiters,
// the replay submitter) under ThreadSanitizer, in host-simulation mode: the
// same admission, batching and completion code runs, batches "run" for a
// modeled time, and no operand is touched.  Several threads submit, poll,
// wait and read statistics at once; a tight byte budget and slot limit make
// admission block and release; destroy drains what is still pending.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <thread>
#include <vector>

#include "mg.h"

static std::atomic<int> failures{0};

static mg_request request(uint64_t id, int64_t n, int algo) {
  const uint64_t base = 0x100000000ull + (id << 26);
  mg_request r{};
  r.dtype = MG_F64;
  r.algo = algo;
  r.p = mg_problem{n, n, n, 1.0, 1.0, reinterpret_cast<void *>(base), n,
                   reinterpret_cast<void *>(base + (1u << 23)), n,
                   reinterpret_cast<void *>(base + (2u << 23)), n};
  return r;
}

int main() {
  mg_server_opts o{};
  o.n_streams = 4;
  o.max_slots = 12;
  o.max_queue = 1 << 16;
  o.max_batch = 8;
  o.hbm_budget_bytes = 64ll << 20;
  o.simulate = 1;
  o.sim_tflops = 40.0;
  o.sim_launch_ns = 5000;
  mg_server *srv = nullptr;
  if (mg_server_create(&o, &srv) != MG_OK) return 2;

  const int kThreads = 4, kPer = 250;
  std::atomic<bool> stop{false};
  std::thread stats_reader([&] {
    while (!stop.load()) {
      mg_server_stats st{};
      if (mg_server_get_stats(srv, &st) != MG_OK) ++failures;
      std::this_thread::yield();
    }
  });
  std::vector<std::thread> workers;
  for (int t = 0; t < kThreads; ++t)
    workers.emplace_back([&, t] {
      std::vector<uint64_t> tickets;
      for (int i = 0; i < kPer; ++i) {
        const uint64_t id = (uint64_t)t * kPer + i;
        const int64_t n = 32 + (int64_t)((id * 97) % 480);
        mg_request r = request(id, n, (id % 10) < 3 ? MG_SPLIT_I8 : MG_NATIVE);
        uint64_t tk = 0;
        if (mg_gemm_submit(srv, &r, &tk) == MG_OK) tickets.push_back(tk);
        else ++failures;
      }
      // half polled to completion, half waited on
      for (size_t i = 0; i < tickets.size(); ++i) {
        mg_result res{};
        int rc;
        if (i % 2 == 0) {
          while ((rc = mg_gemm_poll(srv, tickets[i], &res)) == MG_PENDING) std::this_thread::yield();
        } else {
          rc = mg_gemm_wait(srv, tickets[i], &res);
        }
        if (rc != MG_OK || res.status != MG_OK) ++failures;
      }
    });
  for (auto &w : workers) w.join();

  // open-loop replay from the library's own submitter thread
  const int kReplay = 400;
  std::vector<mg_request> reqs;
  for (int i = 0; i < kReplay; ++i) {
    mg_request r = request(5000 + i, 32 + (i * 53) % 300, i % 4 == 0 ? MG_SPLIT_I8 : MG_NATIVE);
    r.t_arrival_ns = (int64_t)i * 20000;
    reqs.push_back(r);
  }
  std::vector<mg_result> results(kReplay);
  if (mg_server_replay(srv, kReplay, reqs.data(), results.data()) != MG_OK) ++failures;
  for (const mg_result &r : results)
    if (r.status != MG_OK) ++failures;

  // destroy with requests still queued: it must drain them
  for (int i = 0; i < 50; ++i) {
    mg_request r = request(9000 + i, 256, MG_NATIVE);
    uint64_t tk = 0;
    if (mg_gemm_submit(srv, &r, &tk) != MG_OK) ++failures;
  }
  stop = true;
  stats_reader.join();
  mg_server_stats st{};
  mg_server_get_stats(srv, &st);
  if (mg_server_destroy(srv) != MG_OK) ++failures;
  if (st.max_slots_used > o.max_slots || st.max_inflight_bytes > o.hbm_budget_bytes) ++failures;
  std::printf("server under ThreadSanitizer: %lld submitted, %d failures\n",
              (long long)st.submitted, failures.load());
  return failures.load() != 0;
}
