// CPU test of the request server's scheduling core (admission, batching, tickets, failure
// isolation, shutdown) with a test-only executor whose "device work" is the CPU oracle run on a
// helper thread.  Test scaffolding only: the library never uses this executor.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <cstdint>
#include <algorithm>
#include <thread>
#include <vector>

#include "apsort_server_core.h"

extern "C" {
int oracle_sort_u32(const uint32_t* in, uint32_t* out, size_t n);
int oracle_splitters(const uint32_t* sorted, size_t n, int P, uint32_t* splitters);
}

using namespace aps;
using namespace aps::srv;

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::printf("CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c);    \
      g_fail = 1;                                                         \
    }                                                                     \
  } while (0)

class MockExecutor : public Executor {
 public:
  MockExecutor(int slots, size_t cap, int delay_us) : cap_(cap), delay_us_(delay_us), slots_(slots) {
    for (auto& s : slots_) s.done.store(1);
  }
  ~MockExecutor() override {
    for (auto& s : slots_)
      if (s.th.joinable()) s.th.join();
  }
  int num_slots() const override { return (int)slots_.size(); }
  size_t scratch_budget() const override { return cap_; }
  size_t scratch_bytes(const Request& r, bool alone) const override {
    return alone ? r.n * 8 + 1024 : (r.n > 64 ? r.n * 4 : 0);
  }
  ap_status launch_batch(int slot, std::vector<Request*>& reqs, size_t off, size_t len) override {
    size_t bytes = 0;
    for (Request* r : reqs) bytes += Ledger::round_up(scratch_bytes(*r, false));
    if (bytes > Ledger::round_up(len)) len_short++;
    return start(slot, reqs, off, bytes);
  }
  ap_status launch_alone(int slot, Request* r, size_t off, size_t len) override {
    std::vector<Request*> v{r};
    alone_runs++;
    const size_t bytes = Ledger::round_up(scratch_bytes(*r, true));
    if (bytes > Ledger::round_up(len)) len_short++;
    return start(slot, v, off, bytes);
  }
  int query(int slot) override { return slots_[slot].done.load() ? 1 : 0; }

  std::atomic<int> running{0}, max_running{0}, batches{0}, alone_runs{0};
  std::atomic<int> max_batch_seen{0};
  std::atomic<int> overlaps{0}, out_of_arena{0};  // scratch ranges of running work that collide
  std::atomic<int> len_short{0};                   // launches given less scratch than they need
  std::atomic<size_t> max_bytes_in_flight{0};

 private:
  struct S {
    std::atomic<int> done;
    std::thread th;
    size_t off = 0, bytes = 0;
    S() : done(1) {}
    S(const S&) = delete;
  };
  ap_status start(int slot, std::vector<Request*>& reqs, size_t off, size_t bytes) {
    S& s = slots_[slot];
    if (s.th.joinable()) s.th.join();
    // the new range must lie in the arena and miss every range of work still running
    if (off + bytes > cap_) out_of_arena++;
    size_t in_flight = bytes;
    for (int o = 0; o < (int)slots_.size(); ++o) {
      if (o == slot || slots_[o].done.load()) continue;
      const S& t = slots_[o];
      in_flight += t.bytes;
      if (bytes && t.bytes && off < t.off + t.bytes && t.off < off + bytes) overlaps++;
    }
    size_t mb = max_bytes_in_flight.load();
    while (in_flight > mb && !max_bytes_in_flight.compare_exchange_weak(mb, in_flight)) {}
    s.off = off;
    s.bytes = bytes;
    s.done.store(0);
    batches++;
    int b = (int)reqs.size();
    int m = max_batch_seen.load();
    while (b > m && !max_batch_seen.compare_exchange_weak(m, b)) {}
    const int now = ++running;
    int mr = max_running.load();
    while (now > mr && !max_running.compare_exchange_weak(mr, now)) {}
    struct Job { const uint32_t* in; uint32_t* out; size_t n; int P; uint32_t* spl; };
    std::vector<Job> jobs;
    for (Request* r : reqs) jobs.push_back({r->in, r->out, r->n, r->P, r->spl});
    const int delay = delay_us_;
    s.th = std::thread([this, jobs, delay, &s] {
      std::this_thread::sleep_for(std::chrono::microseconds(delay));
      for (const Job& j : jobs) {
        if (j.n) oracle_sort_u32(j.in, j.out, j.n);
        if (j.P > 1 && j.spl) oracle_splitters(j.out, j.n, j.P, j.spl);
      }
      --running;
      s.done.store(1);
    });
    return AP_OK;
  }
  size_t cap_;
  int delay_us_;
  std::vector<S> slots_;
};

struct Buf {
  std::vector<uint32_t> in, out, spl;
};

static void fill(Buf& b, size_t n, int P, std::mt19937& rng) {
  b.in.resize(n);
  for (auto& x : b.in) x = rng();
  b.out.assign(n, 0);
  b.spl.assign(P > 1 ? P - 1 : 1, 0);
}

static bool correct(const Buf& b, int P) {
  std::vector<uint32_t> w = b.in;
  std::sort(w.begin(), w.end());
  if (w != b.out) return false;
  const size_t n = w.size(), q = n / P, r = n % P;
  for (int p = 1; p < P; ++p) {
    const size_t st = p * q + std::min<size_t>(p, r);
    const uint32_t want = st < n ? w[st] : 0xFFFFFFFFu;
    if (b.spl[p - 1] != want) return false;
  }
  return true;
}

static void test_many_requests_two_threads() {
  MockExecutor ex(2, 1 << 20, 200);
  Config c;
  c.max_batch = 16;
  c.alone_min_keys = 20000;
  Server srv(c, &ex);
  const int N = 200;
  std::vector<Buf> bufs(N);
  std::vector<uint64_t> tk(N);
  std::mt19937 rng(1);
  std::vector<size_t> sizes(N);
  std::vector<int> Ps(N);
  for (int i = 0; i < N; ++i) {
    sizes[i] = (i % 17 == 0) ? 30000 : (rng() % 5000);
    Ps[i] = 1 + (int)(rng() % 70);
    fill(bufs[i], sizes[i], Ps[i], rng);
  }
  auto submitter = [&](int lo, int hi) {
    for (int i = lo; i < hi; ++i) {
      ap_status st = srv.submit(bufs[i].in.data(), bufs[i].out.data(), sizes[i], Ps[i], bufs[i].spl.data(), 0, &tk[i]);
      CHECK(st == AP_OK);
    }
  };
  std::thread t1(submitter, 0, N / 2), t2(submitter, N / 2, N);
  t1.join();
  t2.join();
  for (int i = 0; i < N; ++i) CHECK(srv.wait(tk[i], -1) == AP_OK);
  for (int i = 0; i < N; ++i) CHECK(correct(bufs[i], Ps[i]));
  Stats s = srv.stats();
  CHECK(s.completed == (uint64_t)N);
  CHECK(ex.batches.load() < N);       // requests were batched
  CHECK(ex.max_batch_seen.load() > 1);
  CHECK(ex.max_batch_seen.load() <= 16);
  CHECK(ex.alone_runs.load() >= 1);   // long requests ran alone
  CHECK(ex.max_running.load() == 2);  // both slots busy at once
  CHECK(s.latency_us.size() == (size_t)N);
  CHECK(srv.wait(tk[0], 0) == AP_ERR_INVALID);  // forgotten after its final status
}

static void test_budget_queue_and_invalid() {
  MockExecutor ex(1, 4096, 20000);
  Config c;
  c.max_queue = 4;
  Server srv(c, &ex);
  std::vector<uint32_t> big(5000), out(5000);
  uint64_t t = 0;
  CHECK(srv.submit(big.data(), out.data(), 5000, 1, nullptr, 0, &t) == AP_ERR_BUDGET);  // 20000 B > 4096 B
  CHECK(srv.submit(big.data(), out.data(), 10, 0, nullptr, 0, &t) == AP_ERR_INVALID);   // P < 1
  CHECK(srv.submit(big.data(), big.data() + 1, 10, 1, nullptr, 0, &t) == AP_ERR_INVALID);  // partial overlap
  CHECK(srv.submit(nullptr, nullptr, 10, 1, nullptr, 0, &t) == AP_ERR_INVALID);
  // fill the queue while the single slot is busy for 20 ms
  std::vector<std::vector<uint32_t>> in(8, std::vector<uint32_t>(10, 7)), o(8, std::vector<uint32_t>(10));
  std::vector<uint64_t> tk;
  int full = 0;
  for (int i = 0; i < 8; ++i) {
    uint64_t tt = 0;
    ap_status st = srv.submit(in[i].data(), o[i].data(), 10, 1, nullptr, 0, &tt);
    if (st == AP_OK) tk.push_back(tt);
    else if (st == AP_ERR_QUEUE_FULL) full++;
    if (i == 0) std::this_thread::sleep_for(std::chrono::milliseconds(2));  // first one launches
  }
  CHECK(full > 0);
  CHECK(!tk.empty() && srv.wait(tk.back(), 10) == AP_ERR_TIMEOUT);  // still queued behind the slot
  CHECK(srv.poll(tk.back()) == AP_ERR_TIMEOUT);
  for (auto x : tk) CHECK(srv.wait(x, -1) == AP_OK);
}

static void test_injected_fault_isolated() {
  MockExecutor ex(2, 1 << 20, 100);
  Server srv(Config(), &ex);
  std::mt19937 rng(3);
  std::vector<Buf> b(20);
  std::vector<uint64_t> tk(20);
  for (int i = 0; i < 20; ++i) {
    fill(b[i], 300 + i, 4, rng);
    CHECK(srv.submit(b[i].in.data(), b[i].out.data(), b[i].in.size(), 4, b[i].spl.data(), i == 7 ? kInjectFault : 0,
                     &tk[i]) == AP_OK);
  }
  for (int i = 0; i < 20; ++i) {
    const ap_status st = srv.wait(tk[i], -1);
    CHECK(st == (i == 7 ? AP_ERR_DEVICE : AP_OK));
    if (i != 7) CHECK(correct(b[i], 4));
  }
  CHECK(srv.stats().failed == 1);
}

static void test_continuous_batching() {
  MockExecutor ex(2, 1 << 20, 30000);  // 30 ms per batch
  Config c;
  c.max_batch = 64;
  Server srv(c, &ex);
  std::mt19937 rng(5);
  std::vector<Buf> b(30);
  std::vector<uint64_t> tk(30);
  for (int i = 0; i < 10; ++i) {
    fill(b[i], 100, 1, rng);
    CHECK(srv.submit(b[i].in.data(), b[i].out.data(), 100, 1, nullptr, 0, &tk[i]) == AP_OK);
  }
  std::this_thread::sleep_for(std::chrono::milliseconds(5));  // first batch in flight
  for (int i = 10; i < 30; ++i) {
    fill(b[i], 100, 1, rng);
    CHECK(srv.submit(b[i].in.data(), b[i].out.data(), 100, 1, nullptr, 0, &tk[i]) == AP_OK);
  }
  for (int i = 0; i < 30; ++i) CHECK(srv.wait(tk[i], -1) == AP_OK);
  for (int i = 0; i < 30; ++i) CHECK(correct(b[i], 1));
  CHECK(ex.max_running.load() == 2);   // the late arrivals ran while the first batch was running
  CHECK(ex.batches.load() >= 2 && ex.batches.load() <= 3);
}

static void test_shutdown_cancels_queued() {
  MockExecutor ex(1, 1 << 20, 20000);
  Server* srv = new Server(Config(), &ex);
  std::vector<std::vector<uint32_t>> in(5, std::vector<uint32_t>(2000, 1)), o(5, std::vector<uint32_t>(2000));
  uint64_t t = 0;
  CHECK(srv->submit(in[0].data(), o[0].data(), 2000, 1, nullptr, 0, &t) == AP_OK);
  std::this_thread::sleep_for(std::chrono::milliseconds(2));
  for (int i = 1; i < 5; ++i) CHECK(srv->submit(in[i].data(), o[i].data(), 2000, 1, nullptr, 0, &t) == AP_OK);
  Config c2;
  srv->shutdown();
  Stats s = srv->stats();
  CHECK(s.completed == 1);   // the running batch finished
  CHECK(s.cancelled >= 1);   // queued ones were cancelled
  uint64_t t2 = 0;
  CHECK(srv->submit(in[0].data(), o[0].data(), 10, 1, nullptr, 0, &t2) == AP_ERR_CANCELLED);
  delete srv;
}

// The ledger against a brute-force model: a map of 256-byte units, first fit = the lowest run of
// free units that is long enough.
static void test_ledger_against_bitmap() {
  const size_t units = 64, A = Ledger::kAlign;
  Ledger L(units * A + 100);  // the tail below one unit is not usable
  CHECK(L.total() == units * A);
  std::vector<int> owner(units, -1);
  struct Res { size_t off, bytes; };
  std::vector<Res> live;
  std::mt19937 rng(11);
  size_t off = 7;
  CHECK(L.reserve(0, &off) && off == 0 && L.used() == 0);
  CHECK(!L.reserve(units * A + 1, &off) && L.used() == 0);
  for (int step = 0; step < 4000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t bytes = 1 + rng() % (12 * A);
      const size_t k = (bytes + A - 1) / A;
      size_t want = SIZE_MAX;  // brute-force first fit
      for (size_t u = 0; u + k <= units && want == SIZE_MAX; ++u) {
        bool ok = true;
        for (size_t j = u; j < u + k && ok; ++j) ok = owner[j] < 0;
        if (ok) want = u;
      }
      const bool got = L.reserve(bytes, &off);
      CHECK(got == (want != SIZE_MAX));
      if (got) {
        CHECK(off == want * A);
        for (size_t j = want; j < want + k; ++j) owner[j] = 1;
        live.push_back({off, bytes});
      }
    } else {
      const size_t i = rng() % live.size();
      L.release(live[i].off, live[i].bytes);
      for (size_t j = live[i].off / A; j < (live[i].off + live[i].bytes + A - 1) / A; ++j) owner[j] = -1;
      live.erase(live.begin() + i);
    }
    size_t used = 0, run = 0, best = 0;
    for (size_t u = 0; u < units; ++u) {
      used += owner[u] >= 0;
      run = owner[u] < 0 ? run + 1 : 0;
      best = std::max(best, run);
    }
    CHECK(L.used() == used * A);
    CHECK(L.largest_free() == best * A);
    CHECK(L.consistent());
    if (g_fail) return;
  }
  for (const Res& r : live) L.release(r.off, r.bytes);
  CHECK(L.used() == 0 && L.largest_free() == L.total() && L.consistent());
}

// One shared arena: a long request may take most of the budget (more than an even share per
// slot), running work never shares a byte range, and the ledger is whole again at the end.
static void test_shared_budget() {
  const size_t cap = 1 << 20;
  MockExecutor ex(4, cap, 1500);
  Config c;
  c.max_batch = 8;
  c.alone_min_keys = 20000;
  Server srv(c, &ex);
  std::mt19937 rng(7);
  uint64_t t = 0;
  std::vector<uint32_t> huge(140000), hout(140000);
  CHECK(srv.submit(huge.data(), hout.data(), 140000, 1, nullptr, 0, &t) == AP_ERR_BUDGET);  // 1.12 MB > 1 MiB
  const int N = 120;
  std::vector<Buf> b(N);
  std::vector<uint64_t> tk(N);
  std::vector<size_t> n(N);
  for (int i = 0; i < N; ++i) {
    n[i] = (i == 0) ? 100000                        // 0.80 MB: more than a quarter of the budget
         : (i % 10 == 0) ? 30000 + rng() % 30000   // 0.24-0.48 MB, alone
         : (i % 3 == 0) ? 40 : 500 + rng() % 4000;  // no scratch / some scratch, batched
    fill(b[i], n[i], 3, rng);
    CHECK(srv.submit(b[i].in.data(), b[i].out.data(), n[i], 3, b[i].spl.data(), 0, &tk[i]) == AP_OK);
  }
  for (int i = 0; i < N; ++i) CHECK(srv.wait(tk[i], -1) == AP_OK);
  for (int i = 0; i < N; ++i) CHECK(correct(b[i], 3));
  CHECK(ex.overlaps.load() == 0);
  CHECK(ex.out_of_arena.load() == 0);
  CHECK(ex.len_short.load() == 0);
  CHECK(ex.max_bytes_in_flight.load() <= cap);
  CHECK(ex.max_running.load() >= 2);
  CHECK(srv.scratch_in_use() == 0);
  CHECK(srv.ledger_consistent());
  Stats s = srv.stats();
  CHECK(s.scratch_total == cap && s.scratch_peak >= 800000 && s.scratch_peak <= cap);
  CHECK(s.queue_us.size() == (size_t)N && s.latency_us.size() == (size_t)N);
  for (size_t i = 0; i < s.queue_us.size(); ++i) CHECK(s.queue_us[i] >= 0 && s.queue_us[i] <= s.latency_us[i]);
}

// A long request at the head that must wait for scratch is not starved by a stream of short ones:
// while it waits only requests without scratch run, and it starts once running work returns
// enough of the arena.
static void test_long_head_waits_for_scratch() {
  const size_t cap = 1 << 20;
  MockExecutor ex(3, cap, 3000);
  Config c;
  c.max_batch = 4;
  c.alone_min_keys = 20000;
  Server srv(c, &ex);
  std::mt19937 rng(9);
  std::vector<Buf> b(40);
  std::vector<uint64_t> tk(40);
  std::vector<size_t> n(40);
  for (int i = 0; i < 40; ++i) {
    n[i] = (i < 2) ? 70000 : (i % 2 ? 30 : 2000);  // two 0.56 MB requests cannot run together
    fill(b[i], n[i], 2, rng);
    CHECK(srv.submit(b[i].in.data(), b[i].out.data(), n[i], 2, b[i].spl.data(), 0, &tk[i]) == AP_OK);
  }
  for (int i = 0; i < 40; ++i) CHECK(srv.wait(tk[i], -1) == AP_OK);
  for (int i = 0; i < 40; ++i) CHECK(correct(b[i], 2));
  CHECK(ex.overlaps.load() == 0 && ex.out_of_arena.load() == 0);
  CHECK(ex.max_bytes_in_flight.load() <= cap);
  CHECK(srv.scratch_in_use() == 0 && srv.ledger_consistent());
}

int main() {
  test_many_requests_two_threads();
  test_budget_queue_and_invalid();
  test_injected_fault_isolated();
  test_continuous_batching();
  test_shutdown_cancels_queued();
  test_ledger_against_bitmap();
  test_shared_budget();
  test_long_head_waits_for_scratch();
  std::printf(g_fail ? "FAILED\n" : "ALL PASSED\n");
  return g_fail;
}
