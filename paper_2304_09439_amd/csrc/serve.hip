// Continuous-batching server over one context (locc_serve_* in locc.h).
//
// A worker thread owns the GPU side.  Its loop: (1) retire every slot whose
// completion event has fired, copying each request's slice of the slot's
// pinned output buffers into the request and stamping its completion time;
// (2) for every free slot, scan the queue in submission order and take each
// request that fits the slot (pairs, pose updates) and conflicts with
// nothing in flight, in the batch, or left waiting ahead of it (a request
// left behind blocks the objects it touches for the requests after it), copy
// them into the slot's pinned staging buffers and enqueue on the slot's
// stream: H2D copies, the pose scatter, the detect path with the slot's own
// scratch and queue, D2H copies and the completion event; (3) sleep briefly
// when idle.  Slots run on separate
// streams, so a batch that forms while others are on the GPU starts as soon
// as a slot frees up and overlaps with them on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <list>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.h"

using namespace locc;

namespace {

__global__ void scatter_objects(locc_object* table, const int32_t* ids, const locc_object* poses, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) table[ids[k]] = poses[k];
}

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0, Clock::time_point t1) {
  return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Request {
  uint64_t id = 0;
  std::vector<int32_t> upd_ids;
  std::vector<locc_object> upd;
  std::vector<int32_t> pairs;
  std::vector<int32_t> refs;  // distinct objects the pairs read
  std::vector<locc_contact> out;
  std::vector<int32_t> counts;
  Clock::time_point t_submit, t_done;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t* d_pairs = nullptr;
  int32_t* d_upd_ids = nullptr;
  locc_object* d_upd = nullptr;
  locc_contact* d_out = nullptr;
  int32_t* d_counts = nullptr;
  Scratch scratch;
  int32_t* h_pairs = nullptr;
  int32_t* h_upd_ids = nullptr;
  locc_object* h_upd = nullptr;
  locc_contact* h_out = nullptr;
  int32_t* h_counts = nullptr;
  std::vector<Request*> reqs;
  std::vector<int> offs;
  bool busy = false;
};

}  // namespace

struct locc_server {
  locc_ctx* ctx = nullptr;
  locc_serve_config cfg{};
  int32_t batch_pairs = 0;
  bool was_profiling = false;
  locc_object* d_objs = nullptr;
  std::vector<Slot> slots;
  // host state, guarded by mu
  std::mutex mu;
  std::list<Request*> queue;
  std::unordered_map<uint64_t, Request*> reqs;
  int64_t queued_pairs = 0;
  uint64_t next_id = 1;
  locc_serve_stats stats{};
  bool stopping = false;
  // worker-only state
  std::vector<int32_t> upd_busy, ref_busy;  // in-flight / batched requests updating / reading each object
  std::vector<uint8_t> upd_blocked, ref_blocked;  // objects a request left waiting during a scan updates / reads
  std::vector<int32_t> blocked_ids;               // entries to clear after the scan
  std::thread worker;
  std::atomic<int> worker_status{LOCC_OK};
};

namespace {

bool fits_and_free(locc_server* S, const Request* r, int pairs_used, int upd_used) {
  if (pairs_used + (int)r->pairs.size() / 2 > S->batch_pairs) return false;
  if (upd_used + (int)r->upd_ids.size() > S->cfg.max_batch_updates) return false;
  for (int32_t id : r->upd_ids)
    if (S->upd_busy[id] || S->ref_busy[id]) return false;
  for (int32_t id : r->refs)
    if (S->upd_busy[id]) return false;
  return true;
}

// Whether r touches an object a request left waiting ahead of it in this scan
// updates, or updates one it reads: r must not overtake that request.
bool blocked(const locc_server* S, const Request* r) {
  for (int32_t id : r->upd_ids)
    if (S->upd_blocked[id] || S->ref_blocked[id]) return true;
  for (int32_t id : r->refs)
    if (S->upd_blocked[id]) return true;
  return false;
}

void block(locc_server* S, const Request* r) {
  for (int32_t id : r->upd_ids) {
    S->upd_blocked[id] = 1;
    S->blocked_ids.push_back(id);
  }
  for (int32_t id : r->refs) {
    S->ref_blocked[id] = 1;
    S->blocked_ids.push_back(id);
  }
}

// Requests examined per batch at most (bounds the scan when the queue is long).
constexpr int kMaxScan = 1024;

void mark(locc_server* S, const Request* r, int d) {
  for (int32_t id : r->upd_ids) S->upd_busy[id] += d;
  for (int32_t id : r->refs) S->ref_busy[id] += d;
}

locc_status launch_slot(locc_server* S, Slot& sl) {
  locc_ctx* c = S->ctx;
  int np = 0, nu = 0;
  sl.offs.clear();
  for (Request* r : sl.reqs) {
    sl.offs.push_back(np);
    const int rp = (int)r->pairs.size() / 2, ru = (int)r->upd_ids.size();
    std::memcpy(sl.h_pairs + 2 * np, r->pairs.data(), sizeof(int32_t) * 2 * rp);
    std::memcpy(sl.h_upd_ids + nu, r->upd_ids.data(), sizeof(int32_t) * ru);
    std::memcpy(sl.h_upd + nu, r->upd.data(), sizeof(locc_object) * ru);
    np += rp;
    nu += ru;
  }
  sl.offs.push_back(np);
  HIP_TRY(hipMemcpyAsync(sl.d_pairs, sl.h_pairs, sizeof(int32_t) * 2 * np, hipMemcpyHostToDevice, sl.stream));
  if (nu > 0) {
    HIP_TRY(hipMemcpyAsync(sl.d_upd_ids, sl.h_upd_ids, sizeof(int32_t) * nu, hipMemcpyHostToDevice, sl.stream));
    HIP_TRY(hipMemcpyAsync(sl.d_upd, sl.h_upd, sizeof(locc_object) * nu, hipMemcpyHostToDevice, sl.stream));
    hipLaunchKernelGGL(scatter_objects, dim3((nu + 255) / 256), dim3(256), 0, sl.stream, S->d_objs, sl.d_upd_ids,
                       sl.d_upd, nu);
    HIP_TRY(hipGetLastError());
  }
  locc_status st = run_path(c, S->d_objs, S->cfg.max_objects, sl.d_pairs, np, nullptr, sl.d_out, sl.d_counts,
                            nullptr, nullptr, sl.stream, &sl.scratch);
  if (st != LOCC_OK) return st;
  HIP_TRY(hipMemcpyAsync(sl.h_out, sl.d_out, sizeof(locc_contact) * np, hipMemcpyDeviceToHost, sl.stream));
  HIP_TRY(hipMemcpyAsync(sl.h_counts, sl.d_counts, sizeof(int32_t) * 2 * np, hipMemcpyDeviceToHost, sl.stream));
  HIP_TRY(hipEventRecord(sl.done, sl.stream));
  sl.busy = true;
  return LOCC_OK;
}

void retire_slot(locc_server* S, Slot& sl) {
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  for (size_t k = 0; k < sl.reqs.size(); ++k) {
    Request* r = sl.reqs[k];
    const int o = sl.offs[k], n = sl.offs[k + 1] - o;
    r->out.assign(sl.h_out + o, sl.h_out + o + n);
    r->counts.assign(sl.h_counts + 2 * o, sl.h_counts + 2 * (o + n));
    r->t_done = now;
    r->done = true;
    mark(S, r, -1);
    S->stats.completed += 1;
    S->stats.pairs_done += n;
  }
  sl.reqs.clear();
  sl.busy = false;
}

void worker_loop(locc_server* S) {
  (void)hipSetDevice(S->ctx->device);
  Clock::time_point busy_since{};
  bool any_busy = false;
  for (;;) {
    bool progressed = false;
    for (Slot& sl : S->slots)
      if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
        retire_slot(S, sl);
        progressed = true;
      }
    for (Slot& sl : S->slots) {
      if (sl.busy) continue;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        int np = 0, nu = 0, scanned = 0;
        for (auto it = S->queue.begin(); it != S->queue.end() && scanned < kMaxScan; ++scanned) {
          Request* r = *it;
          if (fits_and_free(S, r, np, nu) && !blocked(S, r)) {
            it = S->queue.erase(it);
            mark(S, r, +1);
            np += (int)r->pairs.size() / 2;
            nu += (int)r->upd_ids.size();
            S->queued_pairs -= (int64_t)r->pairs.size() / 2;
            sl.reqs.push_back(r);
            if (!S->cfg.batching) break;
            continue;
          }
          if (!S->cfg.batching) break;  // one request per launch, strictly in order
          block(S, r);
          ++it;
        }
        for (int32_t id : S->blocked_ids) S->upd_blocked[id] = S->ref_blocked[id] = 0;
        S->blocked_ids.clear();
      }
      if (sl.reqs.empty()) continue;
      const locc_status st = launch_slot(S, sl);
      if (st != LOCC_OK) {
        S->worker_status = st;
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        S->queue.clear();
        return;
      }
      std::lock_guard<std::mutex> lk(S->mu);
      S->stats.batches += 1;
      progressed = true;
    }
    bool busy_now = false;
    for (const Slot& sl : S->slots) busy_now |= sl.busy;
    const auto now = Clock::now();
    if (busy_now && !any_busy) busy_since = now;
    if (!busy_now && any_busy) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stats.busy_ms += ms_since(busy_since, now);
    }
    any_busy = busy_now;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stopping && S->queue.empty() && !busy_now) return;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(5));
  }
}

void free_server(locc_server* S) {
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    (void)hipFree(sl.d_pairs);
    (void)hipFree(sl.d_upd_ids);
    (void)hipFree(sl.d_upd);
    (void)hipFree(sl.d_out);
    (void)hipFree(sl.d_counts);
    (void)hipFree(sl.scratch.base);
    (void)hipFree(sl.scratch.queue);
    (void)hipHostFree(sl.h_pairs);
    (void)hipHostFree(sl.h_upd_ids);
    (void)hipHostFree(sl.h_upd);
    (void)hipHostFree(sl.h_out);
    (void)hipHostFree(sl.h_counts);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  (void)hipFree(S->d_objs);
  for (auto& kv : S->reqs) delete kv.second;
  S->ctx->profiling = S->was_profiling;
  delete S;
}

}  // namespace

extern "C" {

locc_status locc_serve_start(locc_ctx* c, const locc_serve_config* cfg, const locc_object* objs, int32_t n_objs,
                             locc_server** out) {
  if (!out) return fail(LOCC_ERR_INVALID_ARG, "null output");
  *out = nullptr;
  if (!c || !cfg || (n_objs > 0 && !objs)) return fail(LOCC_ERR_INVALID_ARG, "null context, config or objects");
  if (!c->d_shapes || !c->have_weights) return fail(LOCC_ERR_NOT_READY, "upload shapes and weights first");
  if (cfg->max_objects <= 0 || n_objs < 0 || n_objs > cfg->max_objects)
    return fail(LOCC_ERR_INVALID_ARG, "object table of %d for %d objects", cfg->max_objects, n_objs);
  if (cfg->slots < 1 || cfg->slots > 4) return fail(LOCC_ERR_INVALID_ARG, "slots=%d: must be 1..4", cfg->slots);
  if (cfg->batching != 0 && cfg->batching != 1) return fail(LOCC_ERR_INVALID_ARG, "batching must be 0 or 1");
  if (cfg->max_batch_pairs < 0 || cfg->max_batch_updates < 0 || cfg->max_queued_pairs < 0)
    return fail(LOCC_ERR_INVALID_ARG, "negative size");
  const int slots = cfg->batching ? cfg->slots : 1;
  const size_t table = sizeof(locc_object) * (size_t)cfg->max_objects;
  const size_t per_update = sizeof(int32_t) + sizeof(locc_object);
  auto slot_bytes = [&](int pairs) {
    return (size_t)pairs * (2 * sizeof(int32_t) + sizeof(locc_contact) + 2 * sizeof(int32_t)) +
           (size_t)cfg->max_batch_updates * per_update + workspace_bytes(c, pairs) + 8 * sizeof(unsigned int);
  };
  int pairs = cfg->max_batch_pairs;
  if (pairs == 0) {  // as many as the budget allows
    int lo = 0, hi = 1 << 24;
    while (lo < hi) {
      const int mid = lo + (hi - lo + 1) / 2;
      if (table + slots * slot_bytes(mid) <= cfg->hbm_budget_bytes) lo = mid;
      else hi = mid - 1;
    }
    pairs = lo;
  }
  if (pairs <= 0 || table + slots * slot_bytes(pairs) > cfg->hbm_budget_bytes)
    return fail(LOCC_ERR_OOM, "budget of %zu bytes does not hold the object table and %d slot(s) of %d pairs",
                cfg->hbm_budget_bytes, slots, pairs);
  HIP_TRY(hipSetDevice(c->device));
  locc_server* S = new locc_server();
  S->ctx = c;
  S->cfg = *cfg;
  S->cfg.slots = slots;
  S->batch_pairs = pairs;
  S->stats.max_batch_pairs = pairs;
  S->was_profiling = c->profiling;
  c->profiling = false;  // the worker thread must not touch the profiling lists
  S->upd_busy.assign(cfg->max_objects, 0);
  S->ref_busy.assign(cfg->max_objects, 0);
  S->upd_blocked.assign(cfg->max_objects, 0);
  S->ref_blocked.assign(cfg->max_objects, 0);
  S->slots.resize(slots);
  hipError_t e = hipMalloc(&S->d_objs, table);
  if (e == hipSuccess && n_objs > 0)
    e = hipMemcpy(S->d_objs, objs, sizeof(locc_object) * n_objs, hipMemcpyHostToDevice);
  const int U = cfg->max_batch_updates > 0 ? cfg->max_batch_updates : 1;
  for (Slot& sl : S->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&sl.d_pairs, sizeof(int32_t) * 2 * pairs);
    if (e == hipSuccess) e = hipMalloc(&sl.d_upd_ids, sizeof(int32_t) * U);
    if (e == hipSuccess) e = hipMalloc(&sl.d_upd, sizeof(locc_object) * U);
    if (e == hipSuccess) e = hipMalloc(&sl.d_out, sizeof(locc_contact) * pairs);
    if (e == hipSuccess) e = hipMalloc(&sl.d_counts, sizeof(int32_t) * 2 * pairs);
    sl.scratch.bytes = workspace_bytes(c, pairs);
    if (e == hipSuccess && sl.scratch.bytes) e = hipMalloc(&sl.scratch.base, sl.scratch.bytes);
    if (e == hipSuccess) e = hipMalloc(&sl.scratch.queue, 2 * sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemset(sl.scratch.queue, 0, 2 * sizeof(unsigned int));
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_pairs, sizeof(int32_t) * 2 * pairs, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_upd_ids, sizeof(int32_t) * U, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_upd, sizeof(locc_object) * U, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_out, sizeof(locc_contact) * pairs, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&sl.h_counts, sizeof(int32_t) * 2 * pairs, hipHostMallocDefault);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_server(S);
    return fail(e == hipErrorOutOfMemory ? LOCC_ERR_OOM : LOCC_ERR_HIP, "server buffers: %s", hipGetErrorString(e));
  }
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return LOCC_OK;
}

locc_status locc_serve_submit(locc_server* S, const int32_t* upd_ids, const locc_object* upd, int32_t n_upd,
                              const int32_t* pairs, int32_t n_pairs, uint64_t* req_id) {
  if (!S || !req_id || n_upd < 0 || n_pairs < 0 || (n_upd > 0 && (!upd_ids || !upd)) || (n_pairs > 0 && !pairs))
    return fail(LOCC_ERR_INVALID_ARG, "null or negative argument");
  if (S->worker_status != LOCC_OK) return fail((locc_status)S->worker_status.load(), "server stopped after an error");
  if (n_pairs > S->batch_pairs || n_upd > S->cfg.max_batch_updates)
    return fail(LOCC_ERR_RANGE, "request of %d pairs / %d updates exceeds one batch (%d / %d)", n_pairs, n_upd,
                S->batch_pairs, S->cfg.max_batch_updates);
  const int32_t M = S->cfg.max_objects;
  Request* r = new Request();
  r->upd_ids.assign(upd_ids, upd_ids + n_upd);
  r->upd.assign(upd, upd + n_upd);
  r->pairs.assign(pairs, pairs + 2 * (size_t)n_pairs);
  for (int32_t id : r->upd_ids)
    if (id < 0 || id >= M) {
      delete r;
      return fail(LOCC_ERR_INVALID_ARG, "update of object %d outside the table of %d", id, M);
    }
  r->refs.reserve(r->pairs.size());
  for (int32_t id : r->pairs)
    if (id >= 0 && id < M) r->refs.push_back(id);  // out-of-range pairs are reported by the kernels
  std::sort(r->refs.begin(), r->refs.end());
  r->refs.erase(std::unique(r->refs.begin(), r->refs.end()), r->refs.end());
  std::sort(r->upd_ids.begin(), r->upd_ids.end());
  if (std::adjacent_find(r->upd_ids.begin(), r->upd_ids.end()) != r->upd_ids.end()) {
    delete r;
    return fail(LOCC_ERR_INVALID_ARG, "an object is updated twice in one request");
  }
  r->upd_ids.assign(upd_ids, upd_ids + n_upd);  // keep the caller's order, paired with upd
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stopping) {
    delete r;
    return fail(LOCC_ERR_INVALID_ARG, "server is stopping");
  }
  if (S->cfg.max_queued_pairs > 0 && S->queued_pairs + n_pairs > S->cfg.max_queued_pairs) {
    delete r;
    return fail(LOCC_ERR_BUSY, "queue holds %lld pairs", (long long)S->queued_pairs);
  }
  r->id = S->next_id++;
  r->t_submit = Clock::now();
  S->queue.push_back(r);
  S->reqs[r->id] = r;
  S->queued_pairs += n_pairs;
  S->stats.submitted += 1;
  *req_id = r->id;
  return LOCC_OK;
}

locc_status locc_serve_poll(locc_server* S, uint64_t id, locc_contact* out, int32_t* counts, int32_t* done,
                            double* latency_ms) {
  if (!S || !done) return fail(LOCC_ERR_INVALID_ARG, "null server or output");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return fail(LOCC_ERR_INVALID_ARG, "unknown request %llu", (unsigned long long)id);
  Request* r = it->second;
  *done = r->done ? 1 : 0;
  if (!r->done) return LOCC_OK;
  if (out) std::memcpy(out, r->out.data(), sizeof(locc_contact) * r->out.size());
  if (counts) std::memcpy(counts, r->counts.data(), sizeof(int32_t) * r->counts.size());
  if (latency_ms) *latency_ms = ms_since(r->t_submit, r->t_done);
  delete r;
  S->reqs.erase(it);
  return LOCC_OK;
}

locc_status locc_serve_get_stats(locc_server* S, locc_serve_stats* st) {
  if (!S || !st) return fail(LOCC_ERR_INVALID_ARG, "null server or output");
  std::lock_guard<std::mutex> lk(S->mu);
  *st = S->stats;
  return LOCC_OK;
}

locc_status locc_serve_stop(locc_server* S) {
  if (!S) return LOCC_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  if (S->worker.joinable()) S->worker.join();
  const int st = S->worker_status;
  free_server(S);
  if (st != LOCC_OK) return fail((locc_status)st, "server worker failed");
  return LOCC_OK;
}

}  // extern "C"
