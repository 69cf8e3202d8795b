// Continuous-batching server over one context (locc_serve_* in locc.h): the
// device side.  serve_core.h holds the host side (request checks, queue,
// conflict-ordered batch formation, worker loop, statistics) and drives the
// HipDevice below, which per slot stages a batch in pinned buffers and
// enqueues on the slot's stream: H2D copies, the pose scatter, the detect
// path with the slot's own scratch and queue, D2H copies and the completion
// event.  Slots run on separate streams, so a batch that forms while others
// are on the GPU starts as soon as a slot frees up and overlaps with them on
// the device.
#include <chrono>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "context.h"
#include "serve_core.h"

using namespace locc;
using serve::Request;

namespace {

__global__ void scatter_objects(locc_object* table, const int32_t* ids, const locc_object* poses, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) table[ids[k]] = poses[k];
}

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
};

// The device side of the server: per slot, pinned staging buffers, device
// buffers, a stream, a completion event and the detect path's own scratch.
struct HipDevice {
  locc_ctx* ctx = nullptr;
  int32_t max_objects = 0;
  locc_object* d_objs = nullptr;
  std::vector<Slot> slot;
  const std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  int slots() const { return (int)slot.size(); }

  locc_status launch(int s, const std::vector<Request*>& batch) {
    Slot& sl = slot[s];
    int np = 0, nu = 0;
    for (Request* r : batch) {
      const int rp = r->n_pairs(), ru = r->n_upd();
      std::memcpy(sl.h_pairs + 2 * np, r->pairs.data(), sizeof(int32_t) * 2 * rp);
      std::memcpy(sl.h_upd_ids + nu, r->upd_ids.data(), sizeof(int32_t) * ru);
      std::memcpy(sl.h_upd + nu, r->upd.data(), sizeof(locc_object) * ru);
      np += rp;
      nu += ru;
    }
    HIP_TRY(hipMemcpyAsync(sl.d_pairs, sl.h_pairs, sizeof(int32_t) * 2 * np, hipMemcpyHostToDevice, sl.stream));
    if (nu > 0) {
      HIP_TRY(hipMemcpyAsync(sl.d_upd_ids, sl.h_upd_ids, sizeof(int32_t) * nu, hipMemcpyHostToDevice, sl.stream));
      HIP_TRY(hipMemcpyAsync(sl.d_upd, sl.h_upd, sizeof(locc_object) * nu, hipMemcpyHostToDevice, sl.stream));
      kernel_launch(scatter_objects, dim3((nu + 255) / 256), dim3(256), 0, sl.stream, d_objs, sl.d_upd_ids,
                         sl.d_upd, nu);
      HIP_TRY(hipGetLastError());
    }
    const locc_status st = run_path(ctx, d_objs, max_objects, sl.d_pairs, np, nullptr, sl.d_out, sl.d_counts,
                                    nullptr, nullptr, sl.stream, &sl.scratch);
    if (st != LOCC_OK) return st;
    HIP_TRY(hipMemcpyAsync(sl.h_out, sl.d_out, sizeof(locc_contact) * np, hipMemcpyDeviceToHost, sl.stream));
    HIP_TRY(hipMemcpyAsync(sl.h_counts, sl.d_counts, sizeof(int32_t) * 2 * np, hipMemcpyDeviceToHost, sl.stream));
    HIP_TRY(hipEventRecord(sl.done, sl.stream));
    return LOCC_OK;
  }

  bool finished(int s) { return hipEventQuery(slot[s].done) == hipSuccess; }

  void collect(int s, const std::vector<Request*>& batch, const std::vector<int>& offs) {
    const Slot& sl = slot[s];
    for (size_t k = 0; k < batch.size(); ++k) {
      const int o = offs[k], n = offs[k + 1] - o;
      batch[k]->out.assign(sl.h_out + o, sl.h_out + o + n);
      batch[k]->counts.assign(sl.h_counts + 2 * o, sl.h_counts + 2 * (o + n));
    }
  }

  double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  void worker_init() { (void)hipSetDevice(ctx->device); }
  void idle_wait() { std::this_thread::sleep_for(std::chrono::microseconds(5)); }

  void release() {
    for (Slot& sl : slot) {
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
    slot.clear();
    (void)hipFree(d_objs);
    d_objs = nullptr;
  }
};

}  // namespace

struct locc_server {
  locc_ctx* ctx = nullptr;
  bool was_profiling = false;
  HipDevice dev;
  std::unique_ptr<serve::Core<HipDevice>> core;
};

namespace {

locc_status report(const serve::Check& ck) {
  if (ck.st == LOCC_OK) return LOCC_OK;
  return fail(ck.st, "%s", ck.msg.c_str());
}

// Joins the worker (if any), then frees the device side.
void free_server(locc_server* S) {
  S->core.reset();
  S->dev.release();
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
  if (pairs == 0) pairs = serve::pairs_for_budget(cfg->hbm_budget_bytes, table, slots, slot_bytes);  // all it allows
  if (pairs <= 0 || table + slots * slot_bytes(pairs) > cfg->hbm_budget_bytes)
    return fail(LOCC_ERR_OOM, "budget of %zu bytes does not hold the object table and %d slot(s) of %d pairs",
                cfg->hbm_budget_bytes, slots, pairs);
  HIP_TRY(hipSetDevice(c->device));
  locc_server* S = new locc_server();
  S->ctx = c;
  S->was_profiling = c->profiling;
  c->profiling = false;  // the worker thread must not touch the profiling lists
  HipDevice& d = S->dev;
  d.ctx = c;
  d.max_objects = cfg->max_objects;
  d.slot.resize(slots);
  hipError_t e = hipMalloc(&d.d_objs, table);
  if (e == hipSuccess && n_objs > 0)
    e = hipMemcpy(d.d_objs, objs, sizeof(locc_object) * n_objs, hipMemcpyHostToDevice);
  const int U = cfg->max_batch_updates > 0 ? cfg->max_batch_updates : 1;
  for (Slot& sl : d.slot) {
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
  serve::Limits L;
  L.max_objects = cfg->max_objects;
  L.batch_pairs = pairs;
  L.max_batch_updates = cfg->max_batch_updates;
  L.max_queued_pairs = cfg->max_queued_pairs;
  L.batching = cfg->batching != 0;
  S->core.reset(new serve::Core<HipDevice>(d, L));
  S->core->start();
  *out = S;
  return LOCC_OK;
}

locc_status locc_serve_submit(locc_server* S, const int32_t* upd_ids, const locc_object* upd, int32_t n_upd,
                              const int32_t* pairs, int32_t n_pairs, uint64_t* req_id) {
  if (!S || !req_id) return fail(LOCC_ERR_INVALID_ARG, "null server or id");
  return report(S->core->submit(upd_ids, upd, n_upd, pairs, n_pairs, req_id));
}

locc_status locc_serve_submit_many(locc_server* S, int32_t n_req, const int32_t* upd_offsets, const int32_t* upd_ids,
                                   const locc_object* upd, const int32_t* pair_offsets, const int32_t* pairs,
                                   uint64_t* req_ids, int32_t* n_accepted) {
  if (!S || !n_accepted) return fail(LOCC_ERR_INVALID_ARG, "null server or count");
  return report(S->core->submit_many(n_req, upd_offsets, upd_ids, upd, pair_offsets, pairs, req_ids, n_accepted));
}

locc_status locc_serve_poll(locc_server* S, uint64_t id, locc_contact* out, int32_t* counts, int32_t* done,
                            double* latency_ms) {
  if (!S) return fail(LOCC_ERR_INVALID_ARG, "null server");
  return report(S->core->poll(id, out, counts, done, latency_ms));
}

locc_status locc_serve_get_stats(locc_server* S, locc_serve_stats* st) {
  if (!S || !st) return fail(LOCC_ERR_INVALID_ARG, "null server or output");
  *st = S->core->stats();
  return LOCC_OK;
}

locc_status locc_serve_stop(locc_server* S) {
  if (!S) return LOCC_OK;
  const locc_status st = S->core->stop();
  free_server(S);
  if (st != LOCC_OK) return fail(st, "server worker failed");
  return LOCC_OK;
}

}  // extern "C"
