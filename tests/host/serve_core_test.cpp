// Host-only unit tests of the server's scheduling core (serve_core.h): request
// checks, conflict tracking, batch formation, slot sizing against a mock
// device-memory budget, busy-time accounting on a fake clock, and the whole
// worker loop against a fake device, single-threaded and with concurrent
// submitters and pollers.  Built and run by tests/test_host_runtime.py with
// the address + undefined-behaviour sanitizers and with the thread sanitizer.
//
// The fake device keeps an object table of its own.  A launch applies the
// batch's pose updates and then evaluates every pair of the batch on the
// table (a request's pairs see its own updates), so the served results show
// which updates each request saw.  The semantics the server promises (every
// request sees the table after its own updates and those of every earlier
// request touching the same objects, as in submission order) means the
// served results equal a sequential replay of the requests in submission
// order; the tests check that, and check on every launch, from scratch, that
// no two requests in flight conflict.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_core.h"

using locc::serve::BusyClock;
using locc::serve::Conflicts;
using locc::serve::Core;
using locc::serve::form_batch;
using locc::serve::Limits;
using locc::serve::make_request;
using locc::serve::pairs_for_budget;
using locc::serve::Request;

static int g_failures = 0;
#define EXPECT(cond)                                                          \
  do {                                                                        \
    if (!(cond)) {                                                            \
      std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
      ++g_failures;                                                           \
    }                                                                         \
  } while (0)

namespace {

locc_object pose(float v) {
  locc_object o{};
  o.p[0] = v;
  o.q[0] = 1.f;
  return o;
}

// The fake device's "detection" of a pair: a value that identifies the poses both objects had.
locc_contact eval_pair(const std::vector<locc_object>& table, int32_t i, int32_t j) {
  locc_contact c{};
  const int32_t n = (int32_t)table.size();
  if (i < 0 || j < 0 || i >= n || j >= n) {
    c.logit = NAN;
    return c;
  }
  c.logit = table[i].p[0];
  c.point[0] = table[j].p[0];
  c.depth = (float)(i * 1000 + j);
  return c;
}

struct Spec {  // what a test submitted
  std::vector<int32_t> upd_ids;
  std::vector<locc_object> upd;
  std::vector<int32_t> pairs;
};

// Replays the requests in id order on a table of its own.
std::map<uint64_t, std::vector<locc_contact>> replay(const std::map<uint64_t, Spec>& reqs, int32_t n_objects) {
  std::vector<locc_object> table(n_objects, pose(-1.f));
  std::map<uint64_t, std::vector<locc_contact>> out;
  for (const auto& kv : reqs) {
    const Spec& s = kv.second;
    for (size_t k = 0; k < s.upd_ids.size(); ++k) table[s.upd_ids[k]] = s.upd[k];
    std::vector<locc_contact> r;
    for (size_t k = 0; k + 1 < s.pairs.size(); k += 2) r.push_back(eval_pair(table, s.pairs[k], s.pairs[k + 1]));
    out[kv.first] = r;
  }
  return out;
}

bool same(const locc_contact& a, const locc_contact& b) {
  auto eq = [](float x, float y) { return (std::isnan(x) && std::isnan(y)) || x == y; };
  return eq(a.logit, b.logit) && eq(a.point[0], b.point[0]) && eq(a.depth, b.depth);
}

// Whether two requests conflict, from their own arrays (independent of Conflicts).
bool conflict(const Request& a, const Request& b, int32_t n) {
  auto touches = [n](const std::vector<int32_t>& ids, int32_t x) {
    for (int32_t v : ids)
      if (v == x && v >= 0 && v < n) return true;
    return false;
  };
  for (int32_t u : a.upd_ids)
    if (touches(b.upd_ids, u) || touches(b.pairs, u)) return true;
  for (int32_t u : b.upd_ids)
    if (touches(a.pairs, u)) return true;
  return false;
}

struct FakeDevice {
  int n_slots = 1;
  int32_t n_objects = 0;
  int64_t tick_us = 5;          // the clock advances by this much whenever the worker idles
  std::atomic<int64_t> now_us{0};
  std::vector<int64_t> finish_us;
  std::vector<std::vector<Request*>> running;
  std::vector<std::vector<locc_contact>> results;  // per slot, the batch's pair results
  std::vector<locc_object> table;
  int fail_at = -1;  // launch number that fails (LOCC_ERR_HIP), -1: none
  // worker-thread log, read after stop
  struct Launch {
    int slot;
    std::vector<uint64_t> ids;
    int pairs, upd;
  };
  std::vector<Launch> log;
  int violations = 0;
  int batch_limit_pairs = 0, batch_limit_upd = 0;
  bool inited = false;

  FakeDevice(int slots, int32_t objects, int limit_pairs, int limit_upd)
      : n_slots(slots), n_objects(objects), finish_us(slots, 0), running(slots), results(slots),
        table(objects, pose(-1.f)), batch_limit_pairs(limit_pairs), batch_limit_upd(limit_upd) {}

  int slots() const { return n_slots; }

  locc_status launch(int s, const std::vector<Request*>& b) {
    if (!inited) ++violations;
    if ((int)log.size() == fail_at) return LOCC_ERR_HIP;
    if (!running[s].empty()) ++violations;  // launched on a busy slot
    // no two requests in flight (this batch and the other slots' batches) conflict
    std::vector<Request*> all(b);
    for (int t = 0; t < n_slots; ++t)
      if (t != s) all.insert(all.end(), running[t].begin(), running[t].end());
    for (size_t x = 0; x < all.size(); ++x)
      for (size_t y = x + 1; y < all.size(); ++y)
        if (conflict(*all[x], *all[y], n_objects)) ++violations;
    int np = 0, nu = 0;
    Launch L{s, {}, 0, 0};
    for (Request* r : b) {
      L.ids.push_back(r->id);
      np += r->n_pairs();
      nu += r->n_upd();
      for (size_t k = 0; k < r->upd_ids.size(); ++k) table[r->upd_ids[k]] = r->upd[k];
    }
    if (np > batch_limit_pairs || nu > batch_limit_upd) ++violations;
    results[s].clear();
    for (Request* r : b)
      for (size_t k = 0; k + 1 < r->pairs.size(); k += 2)
        results[s].push_back(eval_pair(table, r->pairs[k], r->pairs[k + 1]));
    L.pairs = np;
    L.upd = nu;
    log.push_back(L);
    running[s] = b;
    finish_us[s] = now_us.load() + 20 + np;
    return LOCC_OK;
  }
  bool finished(int s) {
    const bool f = now_us.load() >= finish_us[s];
    if (f) running[s].clear();
    return f;
  }
  void collect(int s, const std::vector<Request*>& b, const std::vector<int>& offs) {
    for (size_t k = 0; k < b.size(); ++k) {
      b[k]->out.assign(results[s].begin() + offs[k], results[s].begin() + offs[k + 1]);
      b[k]->counts.assign(2 * (size_t)b[k]->n_pairs(), 7);
    }
  }
  double now_ms() { return now_us.load() * 1e-3; }
  void worker_init() { inited = true; }
  void idle_wait() {
    now_us += tick_us;
    std::this_thread::yield();
  }
};

Request req(std::vector<int32_t> upd_ids, std::vector<int32_t> pairs, int32_t n_objects = 16) {
  Limits L;
  L.max_objects = n_objects;
  L.batch_pairs = 1 << 20;
  L.max_batch_updates = 1 << 20;
  std::vector<locc_object> upd(upd_ids.size(), pose(1.f));
  Request r;
  const auto ck = make_request(L, upd_ids.data(), upd.data(), (int32_t)upd_ids.size(), pairs.data(),
                               (int32_t)(pairs.size() / 2), &r);
  EXPECT(ck.st == LOCC_OK);
  return r;
}

void test_make_request() {
  Limits L;
  L.max_objects = 10;
  L.batch_pairs = 4;
  L.max_batch_updates = 2;
  Request r;
  const int32_t pairs[] = {3, 1, 1, 3, 12, 2, -1, 5};
  const int32_t ids[] = {7, 2};
  const locc_object upd[] = {pose(1), pose(2)};
  EXPECT(make_request(L, ids, upd, 2, pairs, 4, &r).st == LOCC_OK);
  EXPECT((r.refs == std::vector<int32_t>{3, 1, 2, 5}));  // distinct, first appearance, out-of-table left out
  EXPECT((r.upd_ids == std::vector<int32_t>{7, 2}));     // the caller's order, paired with the poses
  EXPECT(r.upd[0].p[0] == 1.f && r.upd[1].p[0] == 2.f);
  EXPECT(r.n_pairs() == 4 && r.pairs.size() == 8);
  EXPECT(make_request(L, ids, upd, 2, pairs, 5, &r).st == LOCC_ERR_RANGE);  // more pairs than a batch
  const int32_t three[] = {1, 2, 3};
  const locc_object upd3[] = {pose(1), pose(2), pose(3)};
  EXPECT(make_request(L, three, upd3, 3, pairs, 1, &r).st == LOCC_ERR_RANGE);
  const int32_t dup[] = {4, 4};
  EXPECT(make_request(L, dup, upd, 2, pairs, 1, &r).st == LOCC_ERR_INVALID_ARG);
  const int32_t out_of_table[] = {10};
  EXPECT(make_request(L, out_of_table, upd, 1, pairs, 1, &r).st == LOCC_ERR_INVALID_ARG);
  const int32_t negative[] = {-1};
  EXPECT(make_request(L, negative, upd, 1, pairs, 1, &r).st == LOCC_ERR_INVALID_ARG);
  EXPECT(make_request(L, nullptr, nullptr, 1, pairs, 1, &r).st == LOCC_ERR_INVALID_ARG);
  EXPECT(make_request(L, ids, upd, 0, nullptr, 1, &r).st == LOCC_ERR_INVALID_ARG);
  EXPECT(make_request(L, ids, upd, -1, pairs, 1, &r).st == LOCC_ERR_INVALID_ARG);
  EXPECT(make_request(L, nullptr, nullptr, 0, nullptr, 0, &r).st == LOCC_OK);  // an empty request is fine
  EXPECT(r.refs.empty() && r.n_pairs() == 0);
}

void test_conflicts() {
  Conflicts cf(16);
  const Request read01 = req({}, {0, 1});
  const Request read12 = req({}, {1, 2});
  const Request upd1 = req({1}, {});
  const Request upd3 = req({3}, {4, 5});
  EXPECT(cf.free_for(read01) && cf.free_for(upd1));
  cf.mark(read01, +1);
  EXPECT(cf.free_for(read12));   // two readers of object 1
  EXPECT(!cf.free_for(upd1));    // an update of an object being read
  EXPECT(cf.free_for(upd3));
  cf.mark(upd3, +1);
  EXPECT(!cf.free_for(req({}, {3, 6})));  // a read of an object being updated
  EXPECT(!cf.free_for(req({3}, {})));     // two updates of one object
  cf.mark(read01, -1);
  EXPECT(cf.free_for(upd1));
  cf.close(upd1);
  EXPECT(cf.closed_for(read12) && cf.closed_for(req({1}, {})) && !cf.closed_for(req({}, {2, 6})));
  cf.end_scan();
  EXPECT(!cf.closed_for(read12));
  cf.mark(upd3, -1);
  EXPECT(cf.idle());
}

std::vector<uint64_t> ids_of(const std::vector<Request*>& b) {
  std::vector<uint64_t> v;
  for (Request* r : b) v.push_back(r->id);
  return v;
}

void test_form_batch() {
  Limits L;
  L.max_objects = 16;
  L.batch_pairs = 10;
  L.max_batch_updates = 3;
  std::vector<Request> rs;
  // 1: reads 0-1; 2: updates 1 (conflicts with 1); 3: reads 1-2 (after 2, which updates 1: waits);
  // 4: reads 5-6 (free); 5: updates 7 (free); 6: reads 7 (conflicts with 5 in the batch)
  rs.push_back(req({}, {0, 1}));
  rs.push_back(req({1}, {}));
  rs.push_back(req({}, {1, 2}));
  rs.push_back(req({}, {5, 6}));
  rs.push_back(req({7}, {}));
  rs.push_back(req({}, {7, 8}));
  for (size_t k = 0; k < rs.size(); ++k) rs[k].id = k + 1;
  std::list<Request*> q;
  for (Request& r : rs) q.push_back(&r);
  Conflicts cf(16);
  auto b1 = form_batch(q, cf, L);
  EXPECT((ids_of(b1) == std::vector<uint64_t>{1, 4, 5}));
  EXPECT(q.size() == 3);
  auto b2 = form_batch(q, cf, L);  // batch 1 still in flight: 2 conflicts with 1, 3 is behind 2, 6 with 5
  EXPECT(b2.empty() && q.size() == 3);
  for (Request* r : b1) cf.mark(*r, -1);
  auto b3 = form_batch(q, cf, L);  // 2 now free; 3 reads what 2 updates; 6 free
  EXPECT((ids_of(b3) == std::vector<uint64_t>{2, 6}));
  for (Request* r : b3) cf.mark(*r, -1);
  auto b4 = form_batch(q, cf, L);
  EXPECT((ids_of(b4) == std::vector<uint64_t>{3}));
  for (Request* r : b4) cf.mark(*r, -1);
  EXPECT(q.empty() && cf.idle());

  // capacity: pairs and updates per batch; a request that does not fit waits and closes its objects
  std::vector<Request> cap;
  cap.push_back(req({}, {0, 1, 0, 2, 0, 3, 0, 4, 0, 5, 0, 6}));   // 6 pairs
  cap.push_back(req({}, {1, 1, 1, 2, 1, 3, 1, 4, 1, 5}));         // 5 pairs: 11 > 10, waits
  cap.push_back(req({9, 10, 11}, {9, 10}));                      // 3 updates, 1 pair
  cap.push_back(req({12}, {}));                                  // a 4th update: waits
  cap.push_back(req({}, {12, 13}));                              // reads 12, which 4 (waiting) updates
  cap.push_back(req({}, {14, 15}));                              // 1 pair, free
  for (size_t k = 0; k < cap.size(); ++k) cap[k].id = k + 1;
  q.clear();
  for (Request& r : cap) q.push_back(&r);
  auto c1 = form_batch(q, cf, L);
  EXPECT((ids_of(c1) == std::vector<uint64_t>{1, 3, 6}));
  for (Request* r : c1) cf.mark(*r, -1);
  auto c2 = form_batch(q, cf, L);
  EXPECT((ids_of(c2) == std::vector<uint64_t>{2, 4}));
  for (Request* r : c2) cf.mark(*r, -1);
  auto c3 = form_batch(q, cf, L);
  EXPECT((ids_of(c3) == std::vector<uint64_t>{5}));
  for (Request* r : c3) cf.mark(*r, -1);

  // without batching: one request per batch, strictly in order (a free request behind a waiting one waits)
  Limits F = L;
  F.batching = false;
  std::vector<Request> fifo;
  fifo.push_back(req({2}, {}));
  fifo.push_back(req({}, {5, 6}));
  for (size_t k = 0; k < fifo.size(); ++k) fifo[k].id = k + 1;
  q.clear();
  for (Request& r : fifo) q.push_back(&r);
  Request busy = req({}, {2, 3});
  cf.mark(busy, +1);
  EXPECT(form_batch(q, cf, F).empty());
  cf.mark(busy, -1);
  auto f1 = form_batch(q, cf, F);
  EXPECT((ids_of(f1) == std::vector<uint64_t>{1}));
  for (Request* r : f1) cf.mark(*r, -1);
  auto f2 = form_batch(q, cf, F);
  EXPECT((ids_of(f2) == std::vector<uint64_t>{2}));
  for (Request* r : f2) cf.mark(*r, -1);

  // the scan stops after max_scan requests
  std::vector<Request> many;
  for (int k = 0; k < 8; ++k) many.push_back(req({}, {k, k + 1}));
  for (size_t k = 0; k < many.size(); ++k) many[k].id = k + 1;
  q.clear();
  for (Request& r : many) q.push_back(&r);
  Request hold = req({}, {0, 0});
  Limits S = L;
  S.batch_pairs = 100;
  auto s1 = form_batch(q, cf, S, 3);
  EXPECT(s1.size() == 3 && q.size() == 5);
  for (Request* r : s1) cf.mark(*r, -1);
  (void)hold;
  EXPECT(cf.idle());

  // a non-empty batch stops looking after max_misses requests passed over in a row
  std::vector<Request> misses;
  misses.push_back(req({0}, {}));                                  // taken
  for (int k = 0; k < 4; ++k) misses.push_back(req({}, {0, 1}));   // read 0, which the batch updates
  misses.push_back(req({}, {5, 6}));                               // free, but after 4 misses
  for (size_t k = 0; k < misses.size(); ++k) misses[k].id = k + 1;
  q.clear();
  for (Request& r : misses) q.push_back(&r);
  auto m1 = form_batch(q, cf, S, 1024, 4);
  EXPECT((ids_of(m1) == std::vector<uint64_t>{1}) && q.size() == 5);
  for (Request* r : m1) cf.mark(*r, -1);
  auto m2 = form_batch(q, cf, S, 1024, 4);  // the misses stop a batch only once it holds a request
  EXPECT((ids_of(m2) == std::vector<uint64_t>{2, 3, 4, 5, 6}) && q.empty());
  for (Request* r : m2) cf.mark(*r, -1);
  EXPECT(cf.idle());
}

void test_budget() {
  auto slot_bytes = [](int p) { return (size_t)100 + (size_t)7 * p; };
  const size_t table = 1000;
  EXPECT(pairs_for_budget(table + 3 * slot_bytes(50), table, 3, slot_bytes) == 50);
  EXPECT(pairs_for_budget(table + 3 * slot_bytes(50) - 1, table, 3, slot_bytes) == 49);
  EXPECT(pairs_for_budget(table + 3 * slot_bytes(50) + 20, table, 3, slot_bytes) == 50);
  EXPECT(pairs_for_budget(table + 3 * slot_bytes(0) - 1, table, 3, slot_bytes) == 0);  // not even empty slots
  EXPECT(pairs_for_budget(table - 1, table, 3, slot_bytes) == 0);                      // not even the table
  EXPECT(pairs_for_budget((size_t)1 << 40, table, 1, slot_bytes, 1000) == 1000);        // the cap
  // a 16 GiB budget with the shape of a BF16 slot at K = 128: 56 B of pairs, contacts and counts plus
  // 4,096 B of rows and 336 B of records per pair, 84,673 objects of 32 B
  auto real = [](int p) { return (size_t)p * (56 + 4096 + 336) + (size_t)4096 * 36 + 32; };
  const size_t budget = (size_t)16 << 30, objs = (size_t)84673 * 32;
  const int p = pairs_for_budget(budget, objs, 3, real);
  EXPECT(p > 0 && objs + 3 * real(p) <= budget && objs + 3 * real(p + 1) > budget);
  EXPECT(pairs_for_budget(budget, objs, 1, real) > 2 * p);
}

void test_busy_clock() {
  BusyClock b;
  b.update(false, 0.0);
  b.update(true, 1.0);
  b.update(true, 2.5);
  b.update(false, 4.0);  // 3 ms busy
  b.update(false, 9.0);
  b.update(true, 10.0);
  b.update(false, 10.25);
  EXPECT(std::fabs(b.total_ms() - 3.25) < 1e-12);
}

template <class C>
void wait_all(C& core, std::map<uint64_t, Spec>& specs, std::map<uint64_t, std::vector<locc_contact>>& got,
              FakeDevice& dev) {
  for (int spin = 0; spin < 50000000 && got.size() < specs.size(); ++spin) {
    for (const auto& kv : specs) {
      if (got.count(kv.first)) continue;
      std::vector<locc_contact> out(kv.second.pairs.size() / 2 + 1);
      std::vector<int32_t> counts(kv.second.pairs.size() + 2);
      int32_t done = 0;
      double lat = -1;
      const auto ck = core.poll(kv.first, out.data(), counts.data(), &done, &lat);
      EXPECT(ck.st == LOCC_OK);
      if (done) {
        out.resize(kv.second.pairs.size() / 2);
        got[kv.first] = out;
        EXPECT(lat >= 0.0);
        for (size_t k = 0; k < kv.second.pairs.size(); ++k) EXPECT(counts[k] == 7);
      }
    }
    std::this_thread::yield();
    (void)dev;
  }
}

void check_results(const std::map<uint64_t, Spec>& specs, const std::map<uint64_t, std::vector<locc_contact>>& got,
                   int32_t n_objects) {
  const auto want = replay(specs, n_objects);
  EXPECT(got.size() == specs.size());
  for (const auto& kv : want) {
    auto it = got.find(kv.first);
    if (it == got.end()) {
      ++g_failures;
      continue;
    }
    EXPECT(it->second.size() == kv.second.size());
    for (size_t k = 0; k < kv.second.size() && k < it->second.size(); ++k) {
      if (!same(it->second[k], kv.second[k])) {
        std::fprintf(stderr, "request %llu pair %zu differs from the replay\n", (unsigned long long)kv.first, k);
        ++g_failures;
        break;
      }
    }
  }
}

// Two versions of 40 requests on disjoint objects, all queued before the worker starts: the first
// versions form one batch, the second versions (each conflicting with its first) the next.
void test_core_two_versions() {
  Limits L;
  L.max_objects = 40;
  L.batch_pairs = 1000;
  L.max_batch_updates = 100;
  FakeDevice dev(1, 40, L.batch_pairs, L.max_batch_updates);
  std::map<uint64_t, Spec> specs;
  {
    Core<FakeDevice> core(dev, L);
    for (int v = 0; v < 2; ++v)
      for (int k = 0; k < 40; ++k) {
        Spec s{{k}, {pose((float)(100 * v + k))}, {k, k, k, k}};
        uint64_t id = 0;
        EXPECT(core.submit(s.upd_ids.data(), s.upd.data(), 1, s.pairs.data(), 2, &id).st == LOCC_OK);
        specs[id] = s;
      }
    core.start();
    std::map<uint64_t, std::vector<locc_contact>> got;
    wait_all(core, specs, got, dev);
    EXPECT(core.stop() == LOCC_OK);
    check_results(specs, got, 40);
    const auto st = core.stats();
    EXPECT(st.submitted == 80 && st.completed == 80 && st.pairs_done == 160);
    EXPECT(st.batches == 2);
    EXPECT(st.busy_ms > 0.0 && st.busy_ms <= dev.now_ms());
    EXPECT(core.idle());
  }
  EXPECT(dev.violations == 0);
  EXPECT(dev.log.size() == 2 && dev.log[0].ids.size() == 40 && dev.log[1].ids.size() == 40);
}

// Strictly one request per launch in submission order without batching.
void test_core_no_batching() {
  Limits L;
  L.max_objects = 8;
  L.batch_pairs = 100;
  L.max_batch_updates = 4;
  L.batching = false;
  FakeDevice dev(1, 8, L.batch_pairs, L.max_batch_updates);
  std::map<uint64_t, Spec> specs;
  Core<FakeDevice> core(dev, L);
  core.start();
  for (int k = 0; k < 30; ++k) {
    Spec s{{k % 8}, {pose((float)k)}, {k % 8, (k + 3) % 8}};
    uint64_t id = 0;
    EXPECT(core.submit(s.upd_ids.data(), s.upd.data(), 1, s.pairs.data(), 1, &id).st == LOCC_OK);
    specs[id] = s;
  }
  std::map<uint64_t, std::vector<locc_contact>> got;
  wait_all(core, specs, got, dev);
  EXPECT(core.stop() == LOCC_OK);
  check_results(specs, got, 8);
  EXPECT(dev.log.size() == 30);
  for (size_t k = 0; k < dev.log.size(); ++k) EXPECT(dev.log[k].ids.size() == 1 && dev.log[k].ids[0] == k + 1);
  EXPECT(dev.violations == 0);
}

// Several submitter threads (single requests and submit_many, retrying on BUSY against a queue limit),
// a poller thread, three slots: every result equals the replay in submission (id) order.
void test_core_concurrent(unsigned seed) {
  const int32_t N = 48;
  Limits L;
  L.max_objects = N;
  L.batch_pairs = 64;
  L.max_batch_updates = 8;
  L.max_queued_pairs = 300;
  FakeDevice dev(3, N, L.batch_pairs, L.max_batch_updates);
  std::mutex spec_mu;
  std::map<uint64_t, Spec> specs;
  std::atomic<int> busy_seen{0};
  {
    Core<FakeDevice> core(dev, L);
    core.start();
    auto submitter = [&](unsigned s) {
      std::mt19937 rng(s);
      std::uniform_int_distribution<int> obj(-1, N);  // -1 and N: out of the table (kept, no conflict)
      for (int k = 0; k < 150;) {
        const int batch = (rng() % 3 == 0) ? 1 + (int)(rng() % 6) : 0;  // 0: a single submit
        std::vector<Spec> group;
        for (int g = 0; g < (batch ? batch : 1); ++g) {
          Spec sp;
          const int nu = (int)(rng() % 3);
          for (int u = 0; u < nu; ++u) {
            int32_t id = (int32_t)(rng() % N);
            if (std::find(sp.upd_ids.begin(), sp.upd_ids.end(), id) != sp.upd_ids.end()) continue;
            sp.upd_ids.push_back(id);
            sp.upd.push_back(pose((float)(s * 100000 + k * 10 + g)));
          }
          const int np = 1 + (int)(rng() % 12);
          for (int p = 0; p < np; ++p) {
            sp.pairs.push_back(obj(rng));
            sp.pairs.push_back(obj(rng));
          }
          group.push_back(sp);
        }
        if (!batch) {
          uint64_t id = 0;
          const Spec& sp = group[0];
          const auto ck = core.submit(sp.upd_ids.data(), sp.upd.data(), (int32_t)sp.upd_ids.size(), sp.pairs.data(),
                                      (int32_t)(sp.pairs.size() / 2), &id);
          if (ck.st == LOCC_ERR_BUSY) {
            ++busy_seen;
            std::this_thread::yield();
            continue;  // the same k again
          }
          EXPECT(ck.st == LOCC_OK);
          std::lock_guard<std::mutex> lk(spec_mu);
          specs[id] = sp;
          ++k;
          continue;
        }
        std::vector<int32_t> uo{0}, po{0}, ui, pr;
        std::vector<locc_object> up;
        for (const Spec& sp : group) {
          ui.insert(ui.end(), sp.upd_ids.begin(), sp.upd_ids.end());
          up.insert(up.end(), sp.upd.begin(), sp.upd.end());
          pr.insert(pr.end(), sp.pairs.begin(), sp.pairs.end());
          uo.push_back((int32_t)ui.size());
          po.push_back((int32_t)(pr.size() / 2));
        }
        std::vector<uint64_t> ids(group.size());
        int32_t acc = -1;
        const auto ck = core.submit_many((int32_t)group.size(), uo.data(), ui.data(), up.data(), po.data(), pr.data(),
                                         ids.data(), &acc);
        EXPECT(ck.st == LOCC_OK || ck.st == LOCC_ERR_BUSY);
        EXPECT(acc >= 0 && acc <= (int32_t)group.size());
        if (ck.st == LOCC_ERR_BUSY) ++busy_seen;
        {
          std::lock_guard<std::mutex> lk(spec_mu);
          for (int32_t g = 0; g < acc; ++g) specs[ids[g]] = group[g];
        }
        k += acc;
        if (ck.st == LOCC_ERR_BUSY) std::this_thread::yield();
      }
    };
    std::vector<std::thread> th;
    for (unsigned t = 0; t < 4; ++t) th.emplace_back(submitter, seed * 7 + t);
    // a poller racing the submitters and the worker
    std::atomic<bool> submitting{true};
    std::map<uint64_t, std::vector<locc_contact>> got;
    std::thread poller([&] {
      while (submitting.load()) {
        std::vector<std::pair<uint64_t, size_t>> todo;
        {
          std::lock_guard<std::mutex> lk(spec_mu);
          for (const auto& kv : specs)
            if (!got.count(kv.first)) todo.push_back({kv.first, kv.second.pairs.size() / 2});
        }
        for (const auto& t : todo) {
          std::vector<locc_contact> out(t.second + 1);
          int32_t done = 0;
          if (core.poll(t.first, out.data(), nullptr, &done, nullptr).st == LOCC_OK && done) {
            out.resize(t.second);
            got[t.first] = out;
          }
        }
        std::this_thread::yield();
      }
    });
    for (auto& t : th) t.join();
    submitting = false;
    poller.join();
    {
      std::map<uint64_t, Spec> rest;
      for (const auto& kv : specs)
        if (!got.count(kv.first)) rest[kv.first] = kv.second;
      std::map<uint64_t, std::vector<locc_contact>> more;
      wait_all(core, rest, more, dev);
      got.insert(more.begin(), more.end());
    }
    EXPECT(core.stop() == LOCC_OK);
    check_results(specs, got, N);
    const auto st = core.stats();
    EXPECT(st.submitted == (int64_t)specs.size() && st.completed == st.submitted);
    int64_t pairs = 0;
    for (const auto& kv : specs) pairs += (int64_t)kv.second.pairs.size() / 2;
    EXPECT(st.pairs_done == pairs);
    EXPECT(st.batches == (int64_t)dev.log.size());
    EXPECT(core.idle());
    // a stopped server refuses new requests
    uint64_t id = 0;
    const int32_t pr[] = {0, 1};
    EXPECT(core.submit(nullptr, nullptr, 0, pr, 1, &id).st == LOCC_ERR_INVALID_ARG);
  }
  EXPECT(dev.violations == 0);
  std::printf("concurrent seed %u: %zu requests in %zu launches, BUSY %d times\n", seed, specs.size(),
              dev.log.size(), busy_seen.load());
}

// A failing launch stops the worker: queued requests are dropped, new ones refused with its status,
// stop() reports it, and nothing leaks.
void test_core_launch_failure() {
  Limits L;
  L.max_objects = 4;
  L.batch_pairs = 2;
  L.max_batch_updates = 1;
  FakeDevice dev(1, 4, L.batch_pairs, L.max_batch_updates);
  dev.fail_at = 2;
  Core<FakeDevice> core(dev, L);
  std::vector<uint64_t> ids;
  for (int k = 0; k < 6; ++k) {
    const int32_t up[] = {k % 4};
    const locc_object po[] = {pose((float)k)};
    const int32_t pr[] = {0, 1, 2, 3};
    uint64_t id = 0;
    EXPECT(core.submit(up, po, 1, pr, 2, &id).st == LOCC_OK);
    ids.push_back(id);
  }
  core.start();
  for (int spin = 0; spin < 50000000; ++spin) {
    const int32_t pr[] = {0, 1};
    uint64_t id = 0;
    if (core.submit(nullptr, nullptr, 0, pr, 1, &id).st == LOCC_ERR_HIP) break;
    std::this_thread::yield();
  }
  EXPECT(core.stop() == LOCC_ERR_HIP);
  int32_t done = 0;
  EXPECT(core.poll(ids[0], nullptr, nullptr, &done, nullptr).st == LOCC_OK && done == 1);
  EXPECT(core.poll(ids[1], nullptr, nullptr, &done, nullptr).st == LOCC_OK && done == 1);
  EXPECT(core.poll(ids[2], nullptr, nullptr, &done, nullptr).st == LOCC_OK && done == 0);  // the failed launch
  EXPECT(core.poll(ids[5], nullptr, nullptr, &done, nullptr).st == LOCC_ERR_INVALID_ARG);  // dropped
  EXPECT(dev.log.size() == 2);
}

void test_submit_many_checks() {
  Limits L;
  L.max_objects = 8;
  L.batch_pairs = 4;
  L.max_batch_updates = 2;
  L.max_queued_pairs = 5;
  FakeDevice dev(1, 8, L.batch_pairs, L.max_batch_updates);
  Core<FakeDevice> core(dev, L);  // not started: everything stays queued
  const int32_t uo[] = {0, 0, 0, 0};
  const int32_t po[] = {0, 2, 4, 6};
  const int32_t pr[] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6};
  uint64_t ids[3] = {};
  int32_t acc = -1;
  auto ck = core.submit_many(3, uo, nullptr, nullptr, po, pr, ids, &acc);
  EXPECT(ck.st == LOCC_ERR_BUSY && acc == 2 && ids[0] == 1 && ids[1] == 2);  // 2 + 2 + 2 > 5
  const int32_t bad_po[] = {0, 2, 1, 3};
  ck = core.submit_many(3, uo, nullptr, nullptr, bad_po, pr, ids, &acc);
  EXPECT(ck.st == LOCC_ERR_INVALID_ARG && acc == 0);
  const int32_t big_po[] = {0, 5};
  ck = core.submit_many(1, uo, nullptr, nullptr, big_po, pr, ids, &acc);
  EXPECT(ck.st == LOCC_ERR_RANGE && acc == 0);
  const int32_t dup_uo[] = {0, 2};
  const int32_t dup_ids[] = {3, 3};
  const locc_object dup_poses[] = {pose(1), pose(2)};
  ck = core.submit_many(1, dup_uo, dup_ids, dup_poses, po, pr, ids, &acc);
  EXPECT(ck.st == LOCC_ERR_INVALID_ARG && acc == 0);
  ck = core.submit_many(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &acc);
  EXPECT(ck.st == LOCC_OK && acc == 0);
  const auto st = core.stats();
  EXPECT(st.submitted == 2);
  core.start();
  int32_t done = 0;
  for (int spin = 0; spin < 50000000 && !done; ++spin) {
    EXPECT(core.poll(ids[1], nullptr, nullptr, &done, nullptr).st == LOCC_OK);
    std::this_thread::yield();
  }
  EXPECT(done == 1);
  EXPECT(core.stop() == LOCC_OK);
}

}  // namespace

int main(int argc, char** argv) {
  const unsigned seeds = argc > 1 ? (unsigned)std::atoi(argv[1]) : 3;
  test_make_request();
  test_conflicts();
  test_form_batch();
  test_budget();
  test_busy_clock();
  test_core_two_versions();
  test_core_no_batching();
  for (unsigned s = 1; s <= seeds; ++s) test_core_concurrent(s);
  test_core_launch_failure();
  test_submit_many_checks();
  if (g_failures) {
    std::fprintf(stderr, "%d failure(s)\n", g_failures);
    return 1;
  }
  std::printf("serve_core: all tests passed\n");
  return 0;
}
