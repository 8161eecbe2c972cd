// Continuous-batching GEMM server.
//
// Threads: one scheduler (admission + batch launch) and one completion
// waiter per stream ("lane").  All shared state is guarded by one mutex.
// A lane holds at most one batch in flight; batches on different lanes run
// concurrently on the device.  Requests admitted while batches run are
// launched together as soon as a lane frees up.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "grouped.h"
#include "split.h"

namespace mg {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

namespace {

struct Req {
  mg_request r;
  uint64_t ticket = 0;
  int64_t bytes = 0;
  mg_result res{};
  bool done = false;
};

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  void *d_buf = nullptr;  // work lists (device)
  size_t d_cap = 0;
  void *h_buf = nullptr;  // pinned staging
  size_t h_cap = 0;
  SplitBatchBuffers sb[2];  // split batches' workspace and staging (INT8, BF16)
  std::vector<Req *> batch;
  int64_t sim_done_ns = 0;  // host simulation: when the batch "completes"
  bool busy = false;      // owns a batch (being launched or in flight)
  bool launched = false;  // event recorded, waiter may wait
  std::thread waiter;
};

int64_t esize_of(int dtype) { return dtype == MG_F64 ? 8 : dtype == MG_F32 ? 4 : 0; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct Server {
  mg_server_opts o{};
  mg_tune_table table{};
  bool has_table = false;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_lane;
  std::deque<Req *> waiting, admitted;
  std::unordered_map<uint64_t, Req *> reqs;
  uint64_t next_ticket = 1;
  int64_t bytes_in = 0;
  int slots = 0;
  std::vector<Lane> lanes;
  std::thread sched;
  bool stop = false, stop_waiters = false;
  mg_server_stats st{};
  int64_t next_batch = 0;
  std::mutex sim_mu;               // host simulation: modeled device backlog
  int64_t sim_device_free_ns = 0;
};

namespace {

int ensure_capacity(Lane &L, size_t bytes) {
  if (bytes <= L.d_cap && bytes <= L.h_cap) return MG_OK;
  size_t cap = std::max<size_t>(bytes, 2 * std::max(L.d_cap, (size_t)1 << 20));
  // The lane's previous batch has completed (busy was false), so its buffers
  // are idle.
  if (L.d_buf) (void)hipFree(L.d_buf);
  if (L.h_buf) (void)hipHostFree(L.h_buf);
  L.d_buf = L.h_buf = nullptr;
  L.d_cap = L.h_cap = 0;
  MG_HIP_TRY(hipMalloc(&L.d_buf, cap));
  MG_HIP_TRY(hipHostMalloc(&L.h_buf, cap, hipHostMallocDefault));
  L.d_cap = L.h_cap = cap;
  return MG_OK;
}

// Host simulation of a batch: modeled duration, no device work.  Batches on
// different lanes share the modeled device, so a batch starts when both its
// lane and the device's backlog allow.
void simulate_batch(Server *S, Lane &L, int64_t batch_id) {
  const int64_t t = now_ns();
  double flops = 0;
  for (Req *q : L.batch) {
    q->res.t_launch_ns = t;
    q->res.batch_id = batch_id;
    q->res.batch_size = (int)L.batch.size();
    const mg_problem &p = q->r.p;
    double f = 2.0 * (double)p.m * (double)p.n * (double)p.k;
    if (q->r.algo != MG_NATIVE) {
      const int sl = split_default_slices(q->r.algo);
      f *= 0.5 * sl * (sl + 1) / 2;
    }
    flops += f;
  }
  const int64_t dur = S->o.sim_launch_ns + (int64_t)(flops / (S->o.sim_tflops * 1e12) * 1e9);
  std::lock_guard<std::mutex> lk(S->sim_mu);
  const int64_t start = std::max(t, S->sim_device_free_ns);
  S->sim_device_free_ns = start + dur;
  L.sim_done_ns = start + dur;
}

// Native requests with m*n*k at least this (1024^3) run as their own launch.
constexpr double kDirectMNK = 1073741824.0;

// Enqueues one batch on lane L (no lock held; L is owned by this batch).
void launch_batch(Server *S, Lane &L, int64_t batch_id) {
  if (S->o.simulate) {
    simulate_batch(S, L, batch_id);
    return;
  }
  const int64_t t = now_ns();
  const int nb = (int)L.batch.size();
  std::vector<mg_problem> p64, p32;
  std::vector<Req *> direct;
  for (Req *q : L.batch) {
    q->res.t_launch_ns = t;
    q->res.batch_id = batch_id;
    q->res.batch_size = nb;
    if (q->r.algo != MG_NATIVE) continue;
    const mg_problem &p = q->r.p;
    // Large problems fill the GPU on their own and run faster with the
    // single-problem work divisions than as 64x64 tiles of the grouped
    // kernel; the choice depends only on the request's own shape.
    if ((double)p.m * (double)p.n * (double)p.k >= kDirectMNK) direct.push_back(q);
    else (q->r.dtype == MG_F64 ? p64 : p32).push_back(p);
  }
  // Order the batch after each request's producer (the caller's writes).
  int rc = MG_OK;
  for (Req *q : L.batch)
    if (q->r.ready_event != nullptr &&
        hipStreamWaitEvent(L.s, static_cast<hipEvent_t>(q->r.ready_event), 0) != hipSuccess)
      rc = MG_ERR_HIP;
  const mg_tune_table *tab = S->has_table ? &S->table : nullptr;
  WorkList w64, w32;
  if (rc == MG_OK) rc = build_worklist(MG_F64, (int64_t)p64.size(), p64.data(), tab, &w64);
  if (rc == MG_OK) rc = build_worklist(MG_F32, (int64_t)p32.size(), p32.data(), tab, &w32);
  const size_t o_t64 = 0;
  const size_t o_t32 = align256(o_t64 + w64.tiles.size());
  const size_t total = align256(o_t32 + w32.tiles.size());
  if (rc == MG_OK && total > 0) rc = ensure_capacity(L, total);
  if (rc == MG_OK && total > 0) {
    unsigned char *h = static_cast<unsigned char *>(L.h_buf);
    auto put = [&](size_t off, const std::vector<unsigned char> &v) {
      if (!v.empty()) std::memcpy(h + off, v.data(), v.size());
    };
    put(o_t64, w64.tiles);
    put(o_t32, w32.tiles);
    if (hipMemcpyAsync(L.d_buf, L.h_buf, total, hipMemcpyHostToDevice, L.s) != hipSuccess)
      rc = MG_ERR_HIP;
    unsigned char *d = static_cast<unsigned char *>(L.d_buf);
    int grid = 1;
    if (rc == MG_OK && w64.ntiles > 0 && (rc = grouped_grid(MG_F64, w64.ntiles, &grid, nullptr)) == MG_OK)
      rc = launch_worklist(MG_F64, d + o_t64, w64.ntiles, grid, L.s);
    if (rc == MG_OK && w32.ntiles > 0 && (rc = grouped_grid(MG_F32, w32.ntiles, &grid, nullptr)) == MG_OK)
      rc = launch_worklist(MG_F32, d + o_t32, w32.ntiles, grid, L.s);
  }
  for (Req *q : L.batch)
    if (q->r.algo == MG_NATIVE && rc != MG_OK) q->res.status = rc;
  for (Req *q : direct) {
    const mg_problem &p = q->r.p;
    const int r2 = gemm_native(q->r.dtype, pick_tile_cfg(q->r.dtype, p.m, p.n, p.k), p.m, p.n,
                               p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C, p.ldc, L.s);
    if (r2 != MG_OK) q->res.status = r2;
  }
  // Split requests: one batched split launch set per algorithm (each result
  // the same bits as the request alone).
  for (const int algo : {MG_SPLIT_I8, MG_SPLIT_BF16}) {
    std::vector<mg_problem> ps;
    for (Req *q : L.batch)
      if (q->r.algo == algo) ps.push_back(q->r.p);
    if (ps.empty()) continue;
    // the lane's own buffers: its previous batch has completed, so they are
    // free, and the batch allocates nothing
    const int r2 = gemm_split_batched(algo, (int64_t)ps.size(), ps.data(), L.s,
                                      &L.sb[algo == MG_SPLIT_BF16 ? 1 : 0]);
    if (r2 != MG_OK)
      for (Req *q : L.batch)
        if (q->r.algo == algo) q->res.status = r2;
  }
  (void)hipEventRecord(L.ev, L.s);
}

void scheduler_loop(Server *S) {
  if (!S->o.simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    while (!S->waiting.empty()) {
      Req *q = S->waiting.front();
      if (S->slots >= S->o.max_slots || S->bytes_in + q->bytes > S->o.hbm_budget_bytes) break;
      S->waiting.pop_front();
      q->res.t_admit_ns = now_ns();
      ++S->slots;
      S->bytes_in += q->bytes;
      S->st.max_inflight_bytes = std::max(S->st.max_inflight_bytes, S->bytes_in);
      S->st.max_slots_used = std::max<int64_t>(S->st.max_slots_used, S->slots);
      S->admitted.push_back(q);
    }
    Lane *free_lane = nullptr;
    for (Lane &L : S->lanes)
      if (!L.busy) {
        free_lane = &L;
        break;
      }
    if (!S->admitted.empty() && free_lane != nullptr) {
      Lane &L = *free_lane;
      L.busy = true;
      const int take = std::min<int>((int)S->admitted.size(), S->o.max_batch);
      L.batch.assign(S->admitted.begin(), S->admitted.begin() + take);
      S->admitted.erase(S->admitted.begin(), S->admitted.begin() + take);
      const int64_t id = S->next_batch++;
      S->st.batches = S->next_batch;
      S->st.max_batch_seen = std::max<int64_t>(S->st.max_batch_seen, take);
      lk.unlock();
      launch_batch(S, L, id);
      lk.lock();
      L.launched = true;
      S->cv_lane.notify_all();
      continue;
    }
    bool idle = S->waiting.empty() && S->admitted.empty();
    for (Lane &L : S->lanes) idle = idle && !L.busy;
    if (S->stop && idle) break;
    S->cv_sched.wait(lk);
  }
}

void waiter_loop(Server *S, Lane *L) {
  if (!S->o.simulate) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_lane.wait(lk, [&] { return L->launched || S->stop_waiters; });
    if (!L->launched) break;
    lk.unlock();
    hipError_t e = hipSuccess;
    if (S->o.simulate) {
      const int64_t wait = L->sim_done_ns - now_ns();
      if (wait > 0) std::this_thread::sleep_for(std::chrono::nanoseconds(wait));
    } else {
      e = hipEventSynchronize(L->ev);
    }
    const int64_t t = now_ns();
    lk.lock();
    for (Req *q : L->batch) {
      q->res.t_done_ns = t;
      if (e != hipSuccess && q->res.status == MG_OK) q->res.status = MG_ERR_HIP;
      if (q->res.status != MG_OK) ++S->st.failed;
      q->done = true;
      --S->slots;
      S->bytes_in -= q->bytes;
      ++S->st.completed;
    }
    L->batch.clear();
    L->launched = false;
    L->busy = false;
    S->cv_sched.notify_all();
    S->cv_done.notify_all();
  }
}

void destroy_lanes(Server *S) {
  for (Lane &L : S->lanes) {
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.s) (void)hipStreamDestroy(L.s);
    if (L.d_buf) (void)hipFree(L.d_buf);
    if (L.h_buf) (void)hipHostFree(L.h_buf);
    for (SplitBatchBuffers &b : L.sb) b.release();
  }
}

}  // namespace

int server_create(const mg_server_opts *o, Server **out) {
  if (o == nullptr || out == nullptr || o->n_streams < 1 || o->n_streams > 8 || o->max_slots < 1 ||
      o->max_queue < 1 || o->max_batch < 1 || o->hbm_budget_bytes <= 0 ||
      (o->simulate && !(o->sim_tflops > 0.0 && o->sim_launch_ns >= 0))) {
    set_error("bad server options");
    return MG_ERR_INVALID_ARG;
  }
  Server *S = new Server();
  S->o = *o;
  if (o->table) {
    S->table = *o->table;
    S->has_table = true;
  }
  S->o.table = nullptr;
  S->lanes.resize((size_t)o->n_streams);
  if (o->simulate) {
    S->sched = std::thread(scheduler_loop, S);
    for (Lane &L : S->lanes) L.waiter = std::thread(waiter_loop, S, &L);
    *out = S;
    return MG_OK;
  }
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    set_error("hipGetDevice failed");
    return MG_ERR_HIP;
  }
  for (Lane &L : S->lanes) {
    if (hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess ||
        ensure_capacity(L, (size_t)1 << 20) != MG_OK) {
      destroy_lanes(S);
      delete S;
      set_error("server resource creation failed");
      return MG_ERR_HIP;
    }
  }
  S->sched = std::thread(scheduler_loop, S);
  for (Lane &L : S->lanes) L.waiter = std::thread(waiter_loop, S, &L);
  *out = S;
  return MG_OK;
}

int server_destroy(Server *S) {
  if (S == nullptr) return MG_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_sched.notify_all();
  S->sched.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop_waiters = true;
  }
  S->cv_lane.notify_all();
  for (Lane &L : S->lanes) L.waiter.join();
  destroy_lanes(S);
  for (auto &kv : S->reqs) delete kv.second;
  delete S;
  return MG_OK;
}

int server_submit(Server *S, const mg_request *r, uint64_t *ticket) {
  const int64_t es = esize_of(r->dtype);
  if (es == 0) {
    set_error("unknown dtype %d", r->dtype);
    return MG_ERR_INVALID_ARG;
  }
  if (r->algo != MG_NATIVE && !((r->algo == MG_SPLIT_I8 || r->algo == MG_SPLIT_BF16) &&
                                r->dtype == MG_F64)) {
    set_error("unsupported dtype/algo %d/%d", r->dtype, r->algo);
    return MG_ERR_UNSUPPORTED;
  }
  const mg_problem &p = r->p;
  int rc = validate_problem("request", p.m, p.n, p.k, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C,
                            p.ldc, es);
  if (rc != MG_OK) return rc;
  int64_t bytes = es * (p.m * p.k + p.k * p.n + p.m * p.n);
  if (r->algo != MG_NATIVE) {
    const int64_t ws =
        split_workspace_bytes(r->algo, split_default_slices(r->algo), p.m, p.n, p.k, false);
    if (ws < 0) return MG_ERR_INVALID_ARG;
    bytes += ws;
  }
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lk(S->mu);
  if (bytes > S->o.hbm_budget_bytes) {
    ++S->st.rejected_memory;
    set_error("request needs %lld bytes, budget is %lld", (long long)bytes,
              (long long)S->o.hbm_budget_bytes);
    return MG_ERR_NO_MEMORY;
  }
  if ((int64_t)S->waiting.size() >= S->o.max_queue) {
    ++S->st.rejected_busy;
    set_error("queue full (%d waiting)", S->o.max_queue);
    return MG_ERR_BUSY;
  }
  Req *q = new Req();
  q->r = *r;
  q->bytes = bytes;
  q->ticket = S->next_ticket++;
  q->res.status = MG_OK;
  q->res.t_submit_ns = t;
  q->res.t_arrival_ns = r->t_arrival_ns ? r->t_arrival_ns : t;
  S->reqs[q->ticket] = q;
  S->waiting.push_back(q);
  ++S->st.submitted;
  *ticket = q->ticket;
  S->cv_sched.notify_all();
  return MG_OK;
}

int server_poll(Server *S, uint64_t ticket, mg_result *out, bool block) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return MG_ERR_NOT_FOUND;
  }
  Req *q = it->second;
  if (!q->done) {
    if (!block) return MG_PENDING;
    S->cv_done.wait(lk, [&] { return q->done; });
  }
  if (out) *out = q->res;
  S->reqs.erase(it);
  delete q;
  return MG_OK;
}

int server_stats(const Server *S, mg_server_stats *out) {
  std::lock_guard<std::mutex> lk(const_cast<Server *>(S)->mu);
  *out = S->st;
  return MG_OK;
}

int server_replay(Server *S, int64_t count, const mg_request *reqs, mg_result *results) {
  std::vector<uint64_t> tickets((size_t)count, 0);
  const int64_t t0 = now_ns();
  std::thread submitter([&] {
    for (int64_t i = 0; i < count; ++i) {
      const int64_t target = t0 + reqs[i].t_arrival_ns;
      int64_t now = now_ns();
      if (target - now > 200000)
        std::this_thread::sleep_for(std::chrono::nanoseconds(target - now - 100000));
      while (now_ns() < target) {
      }
      mg_request r = reqs[i];
      r.t_arrival_ns = target;
      const int rc = server_submit(S, &r, &tickets[(size_t)i]);
      if (rc != MG_OK) {
        tickets[(size_t)i] = 0;
        results[i] = mg_result{};
        results[i].status = rc;
        results[i].t_arrival_ns = target;
        results[i].t_submit_ns = now_ns();
      }
    }
  });
  submitter.join();
  for (int64_t i = 0; i < count; ++i)
    if (tickets[(size_t)i] != 0) {
      const int rc = server_poll(S, tickets[(size_t)i], &results[i], true);
      if (rc != MG_OK) return rc;
    }
  return MG_OK;
}

}  // namespace mg

using namespace mg;

extern "C" {

int64_t mg_now_ns(void) { return now_ns(); }

int mg_server_create(const mg_server_opts *opts, mg_server **out) {
  clear_error();
  if (out) *out = nullptr;
  Server *S = nullptr;
  int rc = server_create(opts, &S);
  if (rc == MG_OK) *out = reinterpret_cast<mg_server *>(S);
  return rc;
}

int mg_server_destroy(mg_server *s) {
  clear_error();
  return server_destroy(reinterpret_cast<Server *>(s));
}

int mg_gemm_submit(mg_server *s, const mg_request *req, uint64_t *ticket) {
  clear_error();
  if (s == nullptr || req == nullptr || ticket == nullptr) {
    set_error("NULL server, request or ticket");
    return MG_ERR_INVALID_ARG;
  }
  return server_submit(reinterpret_cast<Server *>(s), req, ticket);
}

int mg_gemm_poll(mg_server *s, uint64_t ticket, mg_result *out) {
  clear_error();
  if (s == nullptr) {
    set_error("NULL server");
    return MG_ERR_INVALID_ARG;
  }
  return server_poll(reinterpret_cast<Server *>(s), ticket, out, false);
}

int mg_gemm_wait(mg_server *s, uint64_t ticket, mg_result *out) {
  clear_error();
  if (s == nullptr) {
    set_error("NULL server");
    return MG_ERR_INVALID_ARG;
  }
  return server_poll(reinterpret_cast<Server *>(s), ticket, out, true);
}

int mg_server_get_stats(const mg_server *s, mg_server_stats *out) {
  clear_error();
  if (s == nullptr || out == nullptr) {
    set_error("NULL server or out");
    return MG_ERR_INVALID_ARG;
  }
  return server_stats(reinterpret_cast<const Server *>(s), out);
}

int mg_server_replay(mg_server *s, int64_t count, const mg_request *reqs, mg_result *results) {
  clear_error();
  if (s == nullptr || count < 0 || (count > 0 && (reqs == nullptr || results == nullptr))) {
    set_error("bad replay arguments");
    return MG_ERR_INVALID_ARG;
  }
  for (int64_t i = 1; i < count; ++i)
    if (reqs[i].t_arrival_ns < reqs[i - 1].t_arrival_ns) {
      set_error("arrival offsets must be ascending (index %lld)", (long long)i);
      return MG_ERR_INVALID_ARG;
    }
  return server_replay(reinterpret_cast<Server *>(s), count, reqs, results);
}

}  // extern "C"
