// Host side of the continuous-batching server (locc_serve_* in locc.h):
// request checks, the queue, conflict-ordered batch formation, slot sizing
// against a device-memory budget, the worker loop and the statistics.
//
// Nothing here calls HIP.  The device side (staging copies, launches,
// completion queries, result copies) and the clock come from a policy class,
// so the same code runs in serve.hip against the GPU and in host-only unit
// tests against a fake device and a fake clock, built with the address,
// undefined-behaviour and thread sanitizers.
//
// Device policy (all calls but now_ms() come from the worker thread):
//   int slots() const;
//   locc_status launch(int slot, const std::vector<Request*>& batch);
//       stage the batch's updates and pairs, enqueue its work; results later
//   bool finished(int slot);          the slot's last launch has completed
//   void collect(int slot, const std::vector<Request*>& batch, const std::vector<int>& offs);
//       copy the slot's results into the requests (offs: first pair of each, then the total)
//   double now_ms();                  a steady clock, callable from any thread
//   void worker_init();               once, on the worker thread, before anything else
//   void idle_wait();                 the worker found nothing to do
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <list>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "locc.h"

namespace locc {
namespace serve {

struct Request {
  uint64_t id = 0;
  std::vector<int32_t> upd_ids;  // objects updated, in the caller's order (paired with upd)
  std::vector<locc_object> upd;
  std::vector<int32_t> pairs;    // [n][2] object indices
  std::vector<int32_t> refs;     // distinct objects of the table the pairs read
  std::vector<locc_contact> out;
  std::vector<int32_t> counts;
  double t_submit = 0.0, t_done = 0.0;  // ms on the device policy's clock
  bool done = false;
  int n_pairs() const { return (int)(pairs.size() / 2); }
  int n_upd() const { return (int)upd_ids.size(); }
};

struct Limits {
  int32_t max_objects = 0;
  int32_t batch_pairs = 0;        // pairs per batch (one slot's size)
  int32_t max_batch_updates = 0;  // pose updates per batch
  int32_t max_queued_pairs = 0;   // host queue limit in pairs, 0: none
  bool batching = true;           // false: one request per launch, strictly in order
};

// A status with the message the C layer records for locc_last_error.
struct Check {
  locc_status st = LOCC_OK;
  std::string msg;
};

inline Check make_check(locc_status st, const char* fmt, long long a = 0, long long b = 0, long long c = 0,
                        long long d = 0) {
  char buf[256];
  std::snprintf(buf, sizeof buf, fmt, a, b, c, d);
  return Check{st, buf};
}

// Builds a request from the caller's arrays (copied), or says why not:
// INVALID_ARG for null or negative arguments, an update outside the table or
// an object updated twice; RANGE for a request larger than one batch.  Pairs
// naming objects outside the table are kept (the kernels report them) but
// take no part in conflicts.
inline Check make_request(const Limits& L, const int32_t* upd_ids, const locc_object* upd, int32_t n_upd,
                          const int32_t* pairs, int32_t n_pairs, Request* r) {
  if (n_upd < 0 || n_pairs < 0 || (n_upd > 0 && (!upd_ids || !upd)) || (n_pairs > 0 && !pairs))
    return make_check(LOCC_ERR_INVALID_ARG, "null or negative argument");
  if (n_pairs > L.batch_pairs || n_upd > L.max_batch_updates)
    return make_check(LOCC_ERR_RANGE, "request of %lld pairs / %lld updates exceeds one batch (%lld / %lld)", n_pairs,
                      n_upd, L.batch_pairs, L.max_batch_updates);
  for (int32_t k = 0; k < n_upd; ++k)
    if (upd_ids[k] < 0 || upd_ids[k] >= L.max_objects)
      return make_check(LOCC_ERR_INVALID_ARG, "update of object %lld outside the table of %lld", upd_ids[k],
                        L.max_objects);
  // repeated objects found in one pass each, with a per-thread stamp per object and a new stamp per pass
  thread_local std::vector<uint32_t> stamp;
  thread_local uint32_t gen = 0;
  if ((int32_t)stamp.size() < L.max_objects) stamp.assign(L.max_objects, 0u);
  auto next_gen = [&] {
    if (++gen == 0) {  // the stamps wrapped: start over
      std::fill(stamp.begin(), stamp.end(), 0u);
      gen = 1;
    }
  };
  next_gen();
  for (int32_t k = 0; k < n_upd; ++k) {
    if (stamp[upd_ids[k]] == gen) return make_check(LOCC_ERR_INVALID_ARG, "an object is updated twice in one request");
    stamp[upd_ids[k]] = gen;
  }
  r->upd_ids.assign(upd_ids, upd_ids + n_upd);
  r->upd.assign(upd, upd + n_upd);
  r->pairs.assign(pairs, pairs + 2 * (size_t)n_pairs);
  // distinct objects read, in order of first appearance
  next_gen();
  r->refs.clear();
  r->refs.reserve(r->pairs.size());
  for (int32_t id : r->pairs)
    if (id >= 0 && id < L.max_objects && stamp[id] != gen) {
      stamp[id] = gen;
      r->refs.push_back(id);
    }
  return Check{};
}

// Two requests conflict when one updates an object the other reads or
// updates.  Conflicts keeps, per object, how many requests in flight or in
// the forming batch update and read it, and the objects closed during one
// scan of the queue by the requests left waiting.
class Conflicts {
 public:
  explicit Conflicts(int32_t n_objects)
      : upd_busy_(n_objects, 0), ref_busy_(n_objects, 0), upd_closed_(n_objects, 0), ref_closed_(n_objects, 0) {}

  // r conflicts with nothing in flight or in the batch
  bool free_for(const Request& r) const {
    for (int32_t id : r.upd_ids)
      if (upd_busy_[id] || ref_busy_[id]) return false;
    for (int32_t id : r.refs)
      if (upd_busy_[id]) return false;
    return true;
  }
  // r conflicts with a request left waiting earlier in this scan (it must not overtake it)
  bool closed_for(const Request& r) const {
    for (int32_t id : r.upd_ids)
      if (upd_closed_[id] || ref_closed_[id]) return true;
    for (int32_t id : r.refs)
      if (upd_closed_[id]) return true;
    return false;
  }
  void close(const Request& r) {
    for (int32_t id : r.upd_ids) {
      upd_closed_[id] = 1;
      closed_ids_.push_back(id);
    }
    for (int32_t id : r.refs) {
      ref_closed_[id] = 1;
      closed_ids_.push_back(id);
    }
  }
  void end_scan() {
    for (int32_t id : closed_ids_) upd_closed_[id] = ref_closed_[id] = 0;
    closed_ids_.clear();
  }
  // d = +1 when r joins a batch, -1 when its batch completes
  void mark(const Request& r, int d) {
    for (int32_t id : r.upd_ids) upd_busy_[id] += d;
    for (int32_t id : r.refs) ref_busy_[id] += d;
  }
  bool idle() const {
    for (size_t k = 0; k < upd_busy_.size(); ++k)
      if (upd_busy_[k] || ref_busy_[k] || upd_closed_[k] || ref_closed_[k]) return false;
    return closed_ids_.empty();
  }

 private:
  std::vector<int32_t> upd_busy_, ref_busy_;
  std::vector<uint8_t> upd_closed_, ref_closed_;
  std::vector<int32_t> closed_ids_;
};

// Requests examined per batch at most (bounds a scan of a long queue), and
// requests passed over in a row after which a non-empty batch stops looking:
// with a long queue of requests that touch many objects, most requests behind
// a few dozen taken ones conflict with the batch or with one left waiting, and
// examining them costs the worker more than the batch they could still join.
constexpr int kMaxScan = 1024;
constexpr int kMaxMisses = 64;

// Takes the next batch off the queue: scans it in submission order and moves
// each request that fits the batch's remaining pairs and updates, conflicts
// with nothing in flight or in the batch, and does not conflict with a
// request left waiting ahead of it; a request left waiting closes the
// objects it touches for the rest of the scan.  The scan stops after
// max_scan requests, or after max_misses passed over in a row once the batch
// holds one (the requests not examined stay queued, in order).  Without
// batching, the first request if it is free, else nothing.  Marks the taken
// requests in flight.
inline std::vector<Request*> form_batch(std::list<Request*>& queue, Conflicts& cf, const Limits& L,
                                        int max_scan = kMaxScan, int max_misses = kMaxMisses) {
  std::vector<Request*> batch;
  int np = 0, nu = 0, scanned = 0, misses = 0;
  for (auto it = queue.begin(); it != queue.end() && scanned < max_scan; ++scanned) {
    Request* r = *it;
    const bool fits = np + r->n_pairs() <= L.batch_pairs && nu + r->n_upd() <= L.max_batch_updates;
    if (fits && cf.free_for(*r) && !cf.closed_for(*r)) {
      it = queue.erase(it);
      cf.mark(*r, +1);
      np += r->n_pairs();
      nu += r->n_upd();
      batch.push_back(r);
      misses = 0;
      if (!L.batching) break;
      continue;
    }
    if (!L.batching) break;
    if (!batch.empty() && ++misses >= max_misses) break;
    cf.close(*r);
    ++it;
  }
  cf.end_scan();
  return batch;
}

// The largest number of pairs per slot, in [0, cap], for which the object
// table and `slots` slots of slot_bytes(pairs) bytes each fit the budget;
// slot_bytes must not decrease with the pairs.  0 when even an empty slot
// does not fit.
template <class F>
int pairs_for_budget(size_t budget, size_t table, int slots, F slot_bytes, int cap = 1 << 24) {
  auto fits = [&](int pairs) {
    if (table > budget) return false;
    return (size_t)slots * slot_bytes(pairs) <= budget - table;
  };
  if (!fits(0)) return 0;
  int lo = 0, hi = cap;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (fits(mid)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Accumulates the time during which at least one batch is in flight.
class BusyClock {
 public:
  void update(bool busy_now, double now_ms) {
    if (busy_now && !busy_) since_ = now_ms;
    if (!busy_now && busy_) total_ += now_ms - since_;
    busy_ = busy_now;
  }
  double total_ms() const { return total_; }

 private:
  bool busy_ = false;
  double since_ = 0.0, total_ = 0.0;
};

template <class Device>
class Core {
 public:
  Core(Device& dev, const Limits& L) : dev_(dev), L_(L), cf_(L.max_objects), inflight_(dev.slots()) {
    stats_.max_batch_pairs = L.batch_pairs;
  }
  ~Core() {
    stop();
    for (auto& kv : reqs_) delete kv.second;
  }
  Core(const Core&) = delete;
  Core& operator=(const Core&) = delete;

  void start() { worker_ = std::thread([this] { worker_loop(); }); }

  // Queues one request; *id receives its id.  BUSY when the queue limit
  // would be passed, INVALID_ARG once the server stops (or after a worker
  // error, that error).
  Check submit(const int32_t* upd_ids, const locc_object* upd, int32_t n_upd, const int32_t* pairs, int32_t n_pairs,
               uint64_t* id) {
    Request* r = new Request();
    Check ck = make_request(L_, upd_ids, upd, n_upd, pairs, n_pairs, r);
    if (ck.st != LOCC_OK) {
      delete r;
      return ck;
    }
    std::lock_guard<std::mutex> lk(mu_);
    return enqueue(r, id);
  }

  // Queues requests k = 0 .. n - 1 in order, request k holding updates
  // upd_off[k] .. upd_off[k + 1] - 1 and pairs pair_off[k] .. pair_off[k + 1]
  // - 1, under one lock; stops at the first one refused (its status is
  // returned) with *accepted = the number queued.
  Check submit_many(int32_t n, const int32_t* upd_off, const int32_t* upd_ids, const locc_object* upd,
                    const int32_t* pair_off, const int32_t* pairs, uint64_t* ids, int32_t* accepted) {
    *accepted = 0;
    if (n < 0 || (n > 0 && (!upd_off || !pair_off || !ids)))
      return make_check(LOCC_ERR_INVALID_ARG, "null or negative argument");
    for (int32_t k = 0; k < n; ++k)
      if (upd_off[k] < 0 || upd_off[k + 1] < upd_off[k] || pair_off[k] < 0 || pair_off[k + 1] < pair_off[k])
        return make_check(LOCC_ERR_INVALID_ARG, "offsets of request %lld are negative or decreasing", k);
    std::vector<Request*> made(n, nullptr);
    Check ck;
    int32_t ok = 0;
    for (; ok < n; ++ok) {
      Request* r = new Request();
      ck = make_request(L_, upd_ids ? upd_ids + upd_off[ok] : nullptr, upd ? upd + upd_off[ok] : nullptr,
                        upd_off[ok + 1] - upd_off[ok], pairs ? pairs + 2 * (size_t)pair_off[ok] : nullptr,
                        pair_off[ok + 1] - pair_off[ok], r);
      if (ck.st != LOCC_OK) {
        delete r;
        break;
      }
      made[ok] = r;
    }
    std::lock_guard<std::mutex> lk(mu_);
    int32_t k = 0;
    for (; k < ok; ++k) {
      const Check q = enqueue(made[k], ids + k);  // deletes the request it refuses
      if (q.st != LOCC_OK) {
        ck = q;
        for (int32_t j = k + 1; j < ok; ++j) delete made[j];
        break;
      }
    }
    *accepted = k;
    return ck;
  }

  // *done = 1 once request id has completed; then its results are copied
  // out (either pointer may be null) and the request is forgotten.
  Check poll(uint64_t id, locc_contact* out, int32_t* counts, int32_t* done, double* latency_ms) {
    if (!done) return make_check(LOCC_ERR_INVALID_ARG, "null output");
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return make_check(LOCC_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
    Request* r = it->second;
    *done = r->done ? 1 : 0;
    if (!r->done) return Check{};
    if (out) std::copy(r->out.begin(), r->out.end(), out);
    if (counts) std::copy(r->counts.begin(), r->counts.end(), counts);
    if (latency_ms) *latency_ms = r->t_done - r->t_submit;
    delete r;
    reqs_.erase(it);
    return Check{};
  }

  locc_serve_stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    locc_serve_stats s = stats_;
    s.busy_ms = busy_.total_ms();
    return s;
  }

  // Finishes every queued request and joins the worker; returns the
  // worker's status.
  locc_status stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    if (worker_.joinable()) worker_.join();
    return (locc_status)status_.load();
  }

  // No request in flight or waiting and nothing marked (for tests, after stop).
  bool idle() {
    std::lock_guard<std::mutex> lk(mu_);
    return queue_.empty() && cf_.idle();
  }

 private:
  Check enqueue(Request* r, uint64_t* id) {  // mu_ held
    if (status_.load() != LOCC_OK) {
      delete r;
      return make_check((locc_status)status_.load(), "server stopped after an error");
    }
    if (stopping_) {
      delete r;
      return make_check(LOCC_ERR_INVALID_ARG, "server is stopping");
    }
    if (L_.max_queued_pairs > 0 && queued_pairs_ + r->n_pairs() > L_.max_queued_pairs) {
      const long long q = queued_pairs_;
      delete r;
      return make_check(LOCC_ERR_BUSY, "queue holds %lld pairs", q);
    }
    r->id = next_id_++;
    r->t_submit = dev_.now_ms();
    queue_.push_back(r);
    reqs_[r->id] = r;
    queued_pairs_ += r->n_pairs();
    stats_.submitted += 1;
    *id = r->id;
    return Check{};
  }

  void retire(int s) {
    std::vector<Request*>& batch = inflight_[s];
    std::vector<int> offs;
    int np = 0;
    for (Request* r : batch) {
      offs.push_back(np);
      np += r->n_pairs();
    }
    offs.push_back(np);
    dev_.collect(s, batch, offs);  // outside the lock: the requests are the worker's until done is set
    const double now = dev_.now_ms();
    std::lock_guard<std::mutex> lk(mu_);
    for (Request* r : batch) {
      r->t_done = now;
      r->done = true;
      cf_.mark(*r, -1);
      stats_.completed += 1;
      stats_.pairs_done += r->n_pairs();
    }
    batch.clear();
  }

  void fail(locc_status st) {
    std::lock_guard<std::mutex> lk(mu_);
    status_ = st;
    stopping_ = true;
    for (Request* r : queue_) {
      reqs_.erase(r->id);
      delete r;
    }
    queue_.clear();
    queued_pairs_ = 0;
  }

  void worker_loop() {
    dev_.worker_init();
    for (;;) {
      bool progressed = false;
      for (int s = 0; s < (int)inflight_.size(); ++s)
        if (!inflight_[s].empty() && dev_.finished(s)) {
          retire(s);
          progressed = true;
        }
      for (int s = 0; s < (int)inflight_.size(); ++s) {
        if (!inflight_[s].empty()) continue;
        {
          std::lock_guard<std::mutex> lk(mu_);
          inflight_[s] = form_batch(queue_, cf_, L_);
          for (Request* r : inflight_[s]) queued_pairs_ -= r->n_pairs();
        }
        if (inflight_[s].empty()) continue;
        const locc_status st = dev_.launch(s, inflight_[s]);
        if (st != LOCC_OK) {
          // the launched requests stay unfinished (and in reqs_: poll reports them not done)
          fail(st);
          return;
        }
        std::lock_guard<std::mutex> lk(mu_);
        stats_.batches += 1;
        progressed = true;
      }
      bool busy_now = false;
      for (const auto& b : inflight_) busy_now |= !b.empty();
      {
        std::lock_guard<std::mutex> lk(mu_);
        busy_.update(busy_now, dev_.now_ms());
        if (stopping_ && queue_.empty() && !busy_now) return;
      }
      if (!progressed) dev_.idle_wait();
    }
  }

  Device& dev_;
  const Limits L_;
  std::mutex mu_;  // guards everything below except inflight_ (the worker's) and status_ (atomic)
  std::list<Request*> queue_;
  std::unordered_map<uint64_t, Request*> reqs_;
  int64_t queued_pairs_ = 0;
  uint64_t next_id_ = 1;
  locc_serve_stats stats_{};
  BusyClock busy_;
  bool stopping_ = false;
  Conflicts cf_;
  std::vector<std::vector<Request*>> inflight_;
  std::thread worker_;
  std::atomic<int> status_{LOCC_OK};
};

}  // namespace serve
}  // namespace locc
