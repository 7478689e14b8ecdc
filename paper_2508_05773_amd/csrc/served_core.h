// Host-side core of the served form, free of HIP so that it builds and runs on
// the CPU alone (its tests run it under AddressSanitizer, UndefinedBehavior-
// Sanitizer and ThreadSanitizer with a simulated device):
//  - Arena: first-fit sub-allocator over the caller's device arena;
//  - ServedCore: the request queue, the tickets, admission of queued requests
//    into batches by controller state and arena footprint, the stream slots,
//    and the request thread's loop (retire finished batches, admit, launch).
// The device side (launching a batch, querying and retiring it) is a policy
// class the runtime supplies with HIP.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "brmppi.h"

namespace brm {

using Clock = std::chrono::steady_clock;

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// first-fit sub-allocator over the caller's device arena (host bookkeeping of
// offsets only; nothing here touches the memory)
// ---------------------------------------------------------------------------
struct Block {
  char* ptr = nullptr;
  size_t bytes = 0;
};

class Arena {
 public:
  void init(void* base, size_t bytes) {
    base_ = static_cast<char*>(base);
    size_ = bytes;
    used_ = 0;
    free_.clear();
    free_[0] = bytes;
  }
  Block alloc(size_t n) {
    n = round_up(std::max<size_t>(n, 1), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        used_ += n;
        return Block{base_ + off, n};
      }
    }
    return Block{};
  }
  void release(Block& b) {
    if (!b.ptr) return;
    size_t off = (size_t)(b.ptr - base_), len = b.bytes;
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        b = Block{};
        return;
      }
    }
    free_[off] = len;
    b = Block{};
  }
  bool fits(size_t n) const {
    n = round_up(std::max<size_t>(n, 1), 256);
    for (auto& kv : free_)
      if (kv.second >= n) return true;
    return false;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

// ---------------------------------------------------------------------------
// served requests
// ---------------------------------------------------------------------------
// One queued update: a copy of the caller's problem (its obstacle records and
// nominal sequence owned here), and its result once the device is done.
struct Request {
  uint64_t ticket = 0;
  brmppi_problem prob{};
  brmppi_params params{};
  std::vector<brmppi_obstacle> obs;
  std::vector<float> unom;
  std::vector<float> result;
  brmppi_stats st{};
  int status = BRMPPI_PENDING;
  bool done = false;
  size_t footprint = 0;      // device bytes the request adds to a batch
  Clock::time_point t_submit;
};

// copy the caller's problem into r (params: the problem's, or the given
// controller defaults when the pointer is NULL)
inline void copy_problem(Request& r, const brmppi_problem& p, const brmppi_params& params) {
  r.prob = p;
  r.params = params;
  r.prob.params = &r.params;
  r.obs.assign(p.obs, p.obs + p.n_obs);
  r.prob.obs = r.obs.empty() ? nullptr : r.obs.data();
  if (p.u_nom) {
    r.unom.assign(p.u_nom, p.u_nom + 3 * (size_t)p.T);
    r.prob.u_nom = r.unom.data();
  }
}

// A controller's state as admission sees it.
struct SlotState {
  bool busy = false;         // a request of the controller is in flight
  uint32_t warm_T = 0;       // length of its resident warm start (0 = none)
};

constexpr uint32_t kMaxSlots = 4;

// The request queue and the request thread's loop.  Dev supplies the device:
//   using BatchState = ...;                      per-batch device resources
//   int  launch(Batch& b);                       enqueue b on stream slot b.slot; 0, BRMPPI_ENOMEM when its
//                                                packed block does not fit now (nothing was enqueued), or another
//                                                error code (b.state may hold what was enqueued)
//   int  query(Batch& b);                        0 done, 1 running, < 0 error
//   void retire(Batch& b);                       copy results into the requests (result, st, status) and release
//                                                b's device resources
//   void abandon(Batch& b);                      after a failure: wait for what b enqueued, release its resources
//   SlotState& controller(uint32_t id);
//   bool fits(size_t bytes);                     a free block of the arena holds bytes
//   void on_launch(Batch& b), on_complete(Batch& b), trace_push(const char*), trace_pop()
//                                                tracing hooks (a batch's span, the admission pass)
// Every member is guarded by mu; the Dev calls run with mu held.
template <class Dev>
class ServedCore {
 public:
  struct Batch {
    std::vector<Request*> reqs;
    int slot = 0;
    typename Dev::BatchState state{};
  };

  std::mutex mu;
  std::condition_variable cv;

  void configure(uint32_t n_slots, uint32_t max_inflight) {
    n_slots_ = std::min(n_slots, kMaxSlots);
    max_inflight_ = max_inflight ? max_inflight : 4096;
  }

  // ---- API side (mu held by the caller) ----
  // EAGAIN when max_inflight requests are queued or done but unpolled
  int submit(std::unique_ptr<Request> r, uint64_t* ticket) {
    if (n_active_ >= max_inflight_) return BRMPPI_EAGAIN;
    r->ticket = next_ticket_++;
    r->t_submit = Clock::now();
    Request* raw = r.get();
    reqs_[raw->ticket] = std::move(r);
    queue_.push_back(raw);
    ++n_active_;
    *ticket = raw->ticket;
    cv.notify_all();
    return BRMPPI_OK;
  }
  // BRMPPI_PENDING while in flight; ENOTICKET for an unknown or consumed
  // ticket; otherwise copies the result (when u_out is given) and stats,
  // releases the ticket and returns the request's status
  int poll(uint64_t ticket, float* u_out, brmppi_stats* st) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return BRMPPI_ENOTICKET;
    Request* r = it->second.get();
    if (!r->done) return BRMPPI_PENDING;
    if (!u_out) return BRMPPI_EINVAL;
    const int status = r->status;
    if (!r->result.empty()) std::memcpy(u_out, r->result.data(), sizeof(float) * r->result.size());
    if (st) *st = r->st;
    reqs_.erase(it);
    --n_active_;
    return status;
  }
  // poll with a deadline (ETIMEDOUT); takes mu itself
  int wait(uint64_t ticket, float* u_out, brmppi_stats* st, uint32_t timeout_ms) {
    const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      auto it = reqs_.find(ticket);
      if (it == reqs_.end()) return BRMPPI_ENOTICKET;
      if (it->second->done) return poll(ticket, u_out, st);
      const auto now = Clock::now();
      if (now >= deadline) return BRMPPI_ETIMEDOUT;
      nap(lk, std::min<Clock::duration>(deadline - now, std::chrono::milliseconds(1)));
    }
  }
  uint64_t done_count() const { return done_; }
  uint64_t failed_count() const { return failed_; }
  size_t queued() const { return queue_.size(); }
  size_t in_flight() const { return inflight_.size(); }

  // ---- request thread ----
  void start(Dev& dev) {
    running_ = true;
    thread_ = std::thread([this, &dev] { loop(dev); });
  }
  // no new admissions: queued requests fail with ECANCELED, batches in flight
  // drain, the thread ends; then every unpolled ticket is dropped
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu);
      running_ = false;
    }
    cv.notify_all();
    if (thread_.joinable()) thread_.join();
  }

 private:
  // wait on cv for at most d, against a wall-clock deadline (the host C++
  // library waits for a steady-clock deadline with pthread_cond_clockwait,
  // which the host compiler's ThreadSanitizer does not follow through the
  // unlock, and then reports races that do not exist)
  template <class D>
  void nap(std::unique_lock<std::mutex>& lk, D d) {
    cv.wait_until(lk, std::chrono::system_clock::now() + d);
  }

  void fail_request(Request* r, int code) {
    r->status = code;
    r->st.status = code;
    r->done = true;
    ++failed_;
  }
  void fail_batch(Dev& dev, Batch& b, int code) {
    for (Request* r : b.reqs) {
      fail_request(r, code);
      dev.controller(r->prob.controller).busy = false;
    }
    dev.abandon(b);
    slot_busy_[b.slot] = false;
  }
  void retire(Dev& dev, Batch& b) {
    dev.retire(b);
    const auto now = Clock::now();
    for (Request* r : b.reqs) {
      r->st.status = r->status;
      r->st.latency_us = std::chrono::duration<double, std::micro>(now - r->t_submit).count();
      r->done = true;
      SlotState& c = dev.controller(r->prob.controller);
      c.busy = false;
      if (r->status == BRMPPI_OK) c.warm_T = r->prob.T;
      ++done_;
    }
    dev.on_complete(b);
    slot_busy_[b.slot] = false;
  }

  // One admission pass over the queue, in submission order, into batch b:
  //  - a controller gives at most one request per batch and none while it has
  //    one in flight, so that its requests run in order;
  //  - a request without a nominal sequence needs a resident warm start of its
  //    horizon: when its controller is idle and none exists, it fails (ESTATE);
  //  - a request joins while the batch's footprint still fits a free block of
  //    the arena; one that does not fit is skipped, or fails (ENOMEM) when
  //    nothing is in flight and the batch is still empty (no memory can free up).
  // Returns true when a request failed.
  bool admit(Dev& dev, Batch& b) {
    bool failed_any = false;
    size_t budget = 0;
    std::vector<uint32_t> taken;
    auto was_taken = [&](uint32_t c) { return std::find(taken.begin(), taken.end(), c) != taken.end(); };
    for (auto it = queue_.begin(); it != queue_.end() && b.reqs.size() < BRMPPI_MAX_BATCH;) {
      Request* r = *it;
      const uint32_t cid = r->prob.controller;
      SlotState& c = dev.controller(cid);
      if (c.busy || was_taken(cid)) {
        taken.push_back(cid);
        ++it;
        continue;
      }
      if (!r->prob.u_nom && c.warm_T != r->prob.T) {
        fail_request(r, BRMPPI_ESTATE);
        it = queue_.erase(it);
        failed_any = true;
        continue;
      }
      if (!dev.fits(budget + r->footprint)) {
        if (b.reqs.empty() && inflight_.empty()) {
          fail_request(r, BRMPPI_ENOMEM);
          it = queue_.erase(it);
          failed_any = true;
          continue;
        }
        taken.push_back(cid);
        ++it;
        continue;
      }
      budget += r->footprint;
      taken.push_back(cid);
      b.reqs.push_back(r);
      it = queue_.erase(it);
    }
    return failed_any;
  }

  void loop(Dev& dev) {
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      bool progressed = false;
      // retire finished batches (in any order)
      for (size_t i = 0; i < inflight_.size();) {
        const int q = dev.query(inflight_[i]);
        if (q == 0) {
          retire(dev, inflight_[i]);
          inflight_.erase(inflight_.begin() + i);
          progressed = true;
        } else if (q < 0) {
          fail_batch(dev, inflight_[i], BRMPPI_EDEVICE);
          inflight_.erase(inflight_.begin() + i);
          progressed = true;
        } else {
          ++i;
        }
      }
      if (progressed) cv.notify_all();
      // a stopped core runs nothing more: queued requests fail, batches in
      // flight drain
      if (!running_ && !queue_.empty()) {
        for (Request* r : queue_) fail_request(r, BRMPPI_ECANCELED);
        queue_.clear();
        cv.notify_all();
      }
      // admit queued requests into a new batch on a free stream slot
      int slot = -1;
      for (uint32_t k = 0; k < n_slots_; ++k)
        if (!slot_busy_[k]) {
          slot = (int)k;
          break;
        }
      if (slot >= 0 && !queue_.empty()) {
        Batch b;
        b.slot = slot;
        dev.trace_push("brmppi admit");
        const bool failed_any = admit(dev, b);
        dev.trace_pop();
        if (failed_any) {
          progressed = true;
          cv.notify_all();
        }
        if (!b.reqs.empty()) {
          for (Request* r : b.reqs) dev.controller(r->prob.controller).busy = true;
          slot_busy_[slot] = true;
          dev.trace_push("brmppi launch");
          const int rc = dev.launch(b);
          dev.trace_pop();
          if (rc == BRMPPI_OK) {
            dev.on_launch(b);
            inflight_.push_back(std::move(b));
          } else if (rc == BRMPPI_ENOMEM && !inflight_.empty()) {
            // the packed block did not fit (nothing was enqueued): back to the
            // front of the queue, retried once a batch in flight has returned
            // its memory
            for (auto it = b.reqs.rbegin(); it != b.reqs.rend(); ++it) {
              dev.controller((*it)->prob.controller).busy = false;
              queue_.push_front(*it);
            }
            slot_busy_[slot] = false;
          } else {
            fail_batch(dev, b, rc);
            cv.notify_all();
          }
          progressed = true;
        }
      }
      if (!running_ && queue_.empty() && inflight_.empty()) break;
      if (!progressed) {
        if (inflight_.empty() && queue_.empty()) {
          nap(lk, std::chrono::milliseconds(5));
        } else {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::microseconds(20));
          lk.lock();
        }
      }
    }
  }

  uint32_t n_slots_ = 1, max_inflight_ = 4096;
  bool running_ = false;
  uint64_t next_ticket_ = 1;
  std::deque<Request*> queue_;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
  std::vector<Batch> inflight_;
  bool slot_busy_[kMaxSlots] = {false, false, false, false};
  size_t n_active_ = 0;      // queued, running, or done and not yet polled
  uint64_t done_ = 0, failed_ = 0;
  std::thread thread_;
};

}  // namespace brm
