// CPU test of the served form's host core (paper_2508_05773_amd/csrc/served_core.h)
// with a simulated device: batches complete after a pseudo-random delay, and
// each result encodes its ticket, so that every poll can be checked.  Built and
// run by tests/test_served_core_host.py under AddressSanitizer +
// UndefinedBehaviorSanitizer and under ThreadSanitizer.
//
// Checked:
//  - every accepted ticket completes exactly once, with its own result;
//  - a controller's requests run one at a time and complete in submission order;
//  - EAGAIN once max_inflight requests are queued or unpolled;
//  - ESTATE for a request that needs a warm start its controller does not hold;
//  - ENOMEM at admission for a request that fits the arena's size but never its
//    free space (a block held for the whole test), with nothing in flight;
//  - EDEVICE for the requests of a batch whose device work fails;
//  - ECANCELED for requests still queued when the core stops;
//  - the arena returns to its held block only, and no controller stays busy.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "served_core.h"

using namespace brm;

#define CHECK(c)                                                                \
  do {                                                                          \
    if (!(c)) {                                                                 \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);      \
      std::abort();                                                             \
    }                                                                           \
  } while (0)

struct SimDev {
  struct BatchState {
    Block mem;
    Clock::time_point ready;
    bool fault = false;
  };
  Arena* arena = nullptr;
  std::vector<SlotState> ctrl;
  std::vector<std::vector<uint64_t>> completed;   // per controller, in completion order
  std::set<uint32_t> running;                     // controllers with a batch in flight
  std::mt19937 rng{12345};
  int fault_every = 0;                            // every n-th launch fails on the device (0 = never)
  int launches = 0, traces = 0;

  template <class B>
  int launch(B& b) {
    size_t total = 4096;
    for (Request* r : b.reqs) {
      total += r->footprint;
      CHECK(ctrl[r->prob.controller].busy);
      CHECK(running.insert(r->prob.controller).second);   // one request per controller in flight
    }
    b.state.mem = arena->alloc(total);
    if (!b.state.mem.ptr) {
      for (Request* r : b.reqs) running.erase(r->prob.controller);
      return BRMPPI_ENOMEM;
    }
    ++launches;
    b.state.fault = fault_every > 0 && launches % fault_every == 0;
    b.state.ready = Clock::now() + std::chrono::microseconds(rng() % 1500);
    return BRMPPI_OK;
  }
  template <class B>
  int query(B& b) {
    if (Clock::now() < b.state.ready) return 1;
    return b.state.fault ? -1 : 0;
  }
  template <class B>
  void retire(B& b) {
    for (Request* r : b.reqs) {
      r->status = BRMPPI_OK;
      r->result.assign(3 * (size_t)r->prob.T, 0.0f);
      for (size_t k = 0; k < r->result.size(); ++k) r->result[k] = (float)(r->ticket % 100000) + 1e-3f * k;
      r->st.J_min = (float)r->ticket;
      completed[r->prob.controller].push_back(r->ticket);
      running.erase(r->prob.controller);
    }
    arena->release(b.state.mem);
  }
  template <class B>
  void abandon(B& b) {
    for (Request* r : b.reqs) running.erase(r->prob.controller);
    arena->release(b.state.mem);
  }
  SlotState& controller(uint32_t id) { return ctrl[id]; }
  bool fits(size_t bytes) { return arena->fits(bytes + 4096); }
  template <class B>
  void on_launch(B&) { ++traces; }
  template <class B>
  void on_complete(B&) { ++traces; }
  void trace_push(const char*) {}
  void trace_pop() {}
};

static brmppi_problem make_problem(uint32_t controller, uint32_t T, const float* u_nom) {
  brmppi_problem p{};
  p.controller = controller;
  p.S = 1024;
  p.T = T;
  p.u_nom = u_nom;
  p.lambda = 1.0f;
  return p;
}

static std::unique_ptr<Request> make_request(const brmppi_problem& p, size_t footprint) {
  std::unique_ptr<Request> r(new Request());
  copy_problem(*r, p, brmppi_params{});
  r->footprint = footprint;
  return r;
}

// many clients, each with its own controllers, submitting, polling and waiting
static void test_concurrent_clients() {
  constexpr uint32_t kClients = 6, kPerClient = 8, kRequests = 150;
  std::vector<char> mem(64 << 20);
  Arena arena;
  arena.init(mem.data(), mem.size());
  SimDev dev;
  dev.arena = &arena;
  dev.ctrl.resize(kClients * kPerClient);
  dev.completed.resize(kClients * kPerClient);
  ServedCore<SimDev> core;
  core.configure(3, 64);
  core.start(dev);
  std::atomic<int> eagain{0};
  std::vector<std::vector<std::pair<uint32_t, uint64_t>>> submitted(kClients);   // (controller, ticket)
  std::vector<std::thread> th;
  for (uint32_t c = 0; c < kClients; ++c) {
    th.emplace_back([&, c] {
      std::mt19937 rng(77 + c);
      std::vector<float> u(3 * 100, 0.5f);
      std::vector<uint64_t> open;
      auto check_result = [&](uint64_t t, const std::vector<float>& out, const brmppi_stats& st, uint32_t T) {
        CHECK(st.J_min == (float)t);
        for (uint32_t k = 0; k < 3 * T; ++k) CHECK(out[k] == (float)(t % 100000) + 1e-3f * k);
      };
      std::vector<uint32_t> Ts;
      for (uint32_t i = 0; i < kRequests; ++i) {
        const uint32_t ctl = c * kPerClient + (uint32_t)(rng() % kPerClient);
        const uint32_t T = 10 + (uint32_t)(rng() % 90);
        brmppi_problem p = make_problem(ctl, T, u.data());
        uint64_t t = 0;
        int rc;
        while (true) {
          {
            std::lock_guard<std::mutex> lk(core.mu);
            rc = core.submit(make_request(p, 4096 + (rng() % (2 << 20))), &t);
          }
          if (rc != BRMPPI_EAGAIN) break;
          ++eagain;
          // full (the bound is shared by every client): collect this client's
          // oldest open ticket, or let the others collect theirs, then retry
          if (open.empty()) {
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
          }
          std::vector<float> out(300);
          brmppi_stats st{};
          const uint64_t t0 = open.front();
          CHECK(core.wait(t0, out.data(), &st, 20000) == BRMPPI_OK);
          check_result(t0, out, st, Ts.front());
          open.erase(open.begin());
          Ts.erase(Ts.begin());
        }
        CHECK(rc == BRMPPI_OK);
        submitted[c].push_back({ctl, t});
        open.push_back(t);
        Ts.push_back(T);
        // poll the oldest now and then, without blocking
        if (rng() % 3 == 0) {
          std::vector<float> out(300);
          brmppi_stats st{};
          int prc;
          {
            std::lock_guard<std::mutex> lk(core.mu);
            prc = core.poll(open.front(), out.data(), &st);
          }
          if (prc != BRMPPI_PENDING) {
            CHECK(prc == BRMPPI_OK);
            check_result(open.front(), out, st, Ts.front());
            open.erase(open.begin());
            Ts.erase(Ts.begin());
          }
        }
      }
      for (size_t k = 0; k < open.size(); ++k) {
        std::vector<float> out(300);
        brmppi_stats st{};
        CHECK(core.wait(open[k], out.data(), &st, 20000) == BRMPPI_OK);
        check_result(open[k], out, st, Ts[k]);
        // a consumed ticket is gone
        std::lock_guard<std::mutex> lk(core.mu);
        CHECK(core.poll(open[k], out.data(), &st) == BRMPPI_ENOTICKET);
      }
    });
  }
  for (auto& t : th) t.join();
  core.stop();
  // every ticket completed once, per controller in submission order
  for (uint32_t c = 0; c < kClients; ++c) {
    std::vector<std::vector<uint64_t>> per(kPerClient);
    for (auto& st : submitted[c]) per[st.first - c * kPerClient].push_back(st.second);
    for (uint32_t k = 0; k < kPerClient; ++k) CHECK(dev.completed[c * kPerClient + k] == per[k]);
  }
  CHECK(core.done_count() == (uint64_t)kClients * kRequests);
  CHECK(core.failed_count() == 0);
  CHECK(arena.used() == 0);
  for (auto& s : dev.ctrl) CHECK(!s.busy);
  CHECK(eagain.load() > 0);   // the bound of 64 was reached
  std::printf("concurrent clients: %u requests, %d launches, %d EAGAIN retries\n", kClients * kRequests,
              dev.launches, eagain.load());
}

// error paths: ESTATE, ENOMEM at admission, EDEVICE, ECANCELED
static void test_error_paths() {
  std::vector<char> mem(8 << 20);
  Arena arena;
  arena.init(mem.data(), mem.size());
  Block held = arena.alloc(5 << 20);   // the context's persistent allocations
  CHECK(held.ptr);
  SimDev dev;
  dev.arena = &arena;
  dev.ctrl.resize(16);
  dev.completed.resize(16);
  dev.fault_every = 3;
  ServedCore<SimDev> core;
  core.configure(2, 0);
  core.start(dev);
  std::vector<float> u(300, 0.0f);
  auto submit = [&](const brmppi_problem& p, size_t fp) {
    uint64_t t = 0;
    std::lock_guard<std::mutex> lk(core.mu);
    CHECK(core.submit(make_request(p, fp), &t) == BRMPPI_OK);
    return t;
  };
  std::vector<float> out(300);
  brmppi_stats st{};
  // ESTATE: no warm start on controller 0
  uint64_t t = submit(make_problem(0, 20, nullptr), 1024);
  CHECK(core.wait(t, out.data(), &st, 20000) == BRMPPI_ESTATE);
  CHECK(st.status == BRMPPI_ESTATE);
  // a warm start of T = 20 then allows it (the first request may hit a device fault: retry)
  int ok = 0;
  for (int k = 0; k < 3 && !ok; ++k) {
    t = submit(make_problem(0, 20, u.data()), 1024);
    const int rc = core.wait(t, out.data(), &st, 20000);
    CHECK(rc == BRMPPI_OK || rc == BRMPPI_EDEVICE);
    ok = rc == BRMPPI_OK;
  }
  CHECK(ok);
  CHECK(dev.ctrl[0].warm_T == 20);
  int rc = BRMPPI_EDEVICE;
  for (int k = 0; k < 3 && rc == BRMPPI_EDEVICE; ++k) {
    t = submit(make_problem(0, 20, nullptr), 1024);
    rc = core.wait(t, out.data(), &st, 20000);
  }
  CHECK(rc == BRMPPI_OK);
  // a horizon the warm start does not have
  t = submit(make_problem(0, 30, nullptr), 1024);
  CHECK(core.wait(t, out.data(), &st, 20000) == BRMPPI_ESTATE);
  // ENOMEM at admission: fits the arena's 8 MiB, never its 3 MiB of free space
  t = submit(make_problem(1, 20, u.data()), 4 << 20);
  CHECK(core.wait(t, out.data(), &st, 20000) == BRMPPI_ENOMEM);
  // EDEVICE: every third launch fails on the device
  int dev_err = 0, good = 0;
  for (int k = 0; k < 12; ++k) {
    t = submit(make_problem(2 + (k % 4), 20, u.data()), 1024);
    rc = core.wait(t, out.data(), &st, 20000);
    CHECK(rc == BRMPPI_OK || rc == BRMPPI_EDEVICE);
    (rc == BRMPPI_OK ? good : dev_err)++;
  }
  CHECK(dev_err > 0 && good > 0);
  // ETIMEDOUT, then the result once it is there
  dev.fault_every = 0;
  t = submit(make_problem(9, 20, u.data()), 1024);
  rc = core.wait(t, out.data(), &st, 0);
  CHECK(rc == BRMPPI_ETIMEDOUT || rc == BRMPPI_OK);
  if (rc == BRMPPI_ETIMEDOUT) CHECK(core.wait(t, out.data(), &st, 20000) == BRMPPI_OK);
  // ECANCELED: a long queue on one controller, stopped at once
  std::vector<uint64_t> tickets;
  for (int k = 0; k < 40; ++k) tickets.push_back(submit(make_problem(10, 20, u.data()), 1024));
  core.stop();
  int canceled = 0, done = 0;
  for (uint64_t tk : tickets) {
    std::lock_guard<std::mutex> lk(core.mu);
    rc = core.poll(tk, out.data(), &st);
    CHECK(rc == BRMPPI_OK || rc == BRMPPI_ECANCELED);
    (rc == BRMPPI_OK ? done : canceled)++;
  }
  CHECK(canceled > 0);
  arena.release(held);
  CHECK(arena.used() == 0);
  for (auto& s : dev.ctrl) CHECK(!s.busy);
  std::printf("error paths: %d device failures, %d completed, %d canceled of 40\n", dev_err, done, canceled);
}

// the allocator alone: random alloc/release against a reference model
static void test_arena() {
  std::vector<char> mem(1 << 20);
  Arena a;
  a.init(mem.data(), mem.size());
  std::mt19937 rng(5);
  std::vector<Block> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 2) {
      Block b = a.alloc(1 + rng() % 20000);
      if (b.ptr) {
        for (auto& o : live) CHECK(b.ptr + b.bytes <= o.ptr || o.ptr + o.bytes <= b.ptr);   // no overlap
        CHECK(b.ptr >= mem.data() && b.ptr + b.bytes <= mem.data() + mem.size());
        live.push_back(b);
      }
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k]);
      live.erase(live.begin() + k);
    }
    size_t used = 0;
    for (auto& o : live) used += o.bytes;
    CHECK(a.used() == used);
  }
  for (auto& b : live) a.release(b);
  CHECK(a.used() == 0);
  CHECK(a.fits(mem.size()));   // fully coalesced again
  std::printf("arena: ok\n");
}

int main() {
  test_arena();
  test_error_paths();
  test_concurrent_clients();
  std::printf("served core: all checks passed\n");
  return 0;
}
