// Scheduling core of the sort-request server: tickets, a bounded arrival queue, admission under a
// memory budget, continuous batching into launches on a few streams (slots), completion and
// latency statistics.
//
// The core knows nothing about HIP: device work goes through the Executor interface (the HIP
// executor lives in apsort_server.hip).  A slot is one stream; at most one batch (or one large
// request) runs on a slot at a time, so the number of slots bounds the batches in flight.  Scratch
// memory comes from one arena shared by all slots and is kept as a ledger: each unit of work
// reserves the byte range it needs when it is launched and returns it when it completes, so one
// large request may use most of the budget while small batches use little.  Requests that arrive
// while batches run wait in the queue and join the next batch formed on a slot that frees up.
#pragma once

#include <stddef.h>
#include <stdint.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "apsort.h"

namespace aps {
namespace srv {

inline uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr unsigned kInjectFault = 1u;  // test hook: the request fails with AP_ERR_DEVICE, alone

struct Request {
  uint64_t ticket = 0;
  const uint32_t* in = nullptr;
  uint32_t* out = nullptr;
  size_t n = 0;
  int P = 1;
  uint32_t* spl = nullptr;
  unsigned flags = 0;
  uint64_t t_submit = 0, t_launch = 0, t_done = 0;
  int status = -1;  // -1 pending/running, else an ap_status
};

// First-fit ledger of the scratch arena: reservations are byte ranges of [0, total), in units of
// kAlign bytes; a released range merges with free neighbours.  Not thread-safe (the server holds
// its lock around every call).
class Ledger {
 public:
  static constexpr size_t kAlign = 256;
  explicit Ledger(size_t total = 0) { reset(total); }

  void reset(size_t total) {
    total_ = total / kAlign * kAlign;
    free_.clear();
    if (total_) free_[0] = total_;
    used_ = peak_ = 0;
  }
  static size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  size_t total() const { return total_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

  // Reserves `bytes` (rounded up to kAlign) at the lowest offset where they fit; false (and
  // nothing reserved) when no free range is large enough.  Zero bytes always succeed at offset 0.
  bool reserve(size_t bytes, size_t* off) {
    bytes = round_up(bytes);
    *off = 0;
    if (bytes == 0) return true;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }

  // Returns a range that reserve() gave out (same size argument).
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    if (bytes == 0) return;
    size_t start = off, len = bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
    used_ -= bytes;
  }

  // Free ranges ordered, in bounds, neither overlapping nor touching, and summing with the
  // reserved bytes to the total.
  bool consistent() const {
    size_t end = 0, sum = 0;
    bool first = true;
    for (const auto& kv : free_) {
      if (kv.second == 0 || kv.first % kAlign || kv.second % kAlign) return false;
      if (!first && kv.first <= end) return false;  // overlapping or touching the previous range
      end = kv.first + kv.second;
      if (end > total_) return false;
      sum += kv.second;
      first = false;
    }
    return sum + used_ == total_;
  }

 private:
  size_t total_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

// Device side of the server.  All calls come from the scheduler thread.
class Executor {
 public:
  virtual ~Executor() {}
  virtual int num_slots() const = 0;
  // Scratch bytes a request needs (batched or alone); more than scratch_budget() means it can
  // never run.
  virtual size_t scratch_bytes(const Request& r, bool alone) const = 0;
  // Size of the scratch arena that all slots share.
  virtual size_t scratch_budget() const = 0;
  // Enqueue the batch on the slot, with scratch at [scratch_off, scratch_off + scratch_len) of the
  // arena (what scratch_bytes() asked for when the work was admitted).  Returns AP_OK or an error
  // (then every request of the batch fails with AP_ERR_DEVICE).
  virtual ap_status launch_batch(int slot, std::vector<Request*>& reqs, size_t scratch_off, size_t scratch_len) = 0;
  virtual ap_status launch_alone(int slot, Request* r, size_t scratch_off, size_t scratch_len) = 0;
  // 1 = the slot's work completed, 0 = still running, < 0 = the device reported an error.
  virtual int query(int slot) = 0;
  virtual void thread_init() {}
};

struct Config {
  size_t budget = (size_t)64 << 30;
  int num_streams = 4;
  int max_batch = 256;
  int max_queue = 1 << 16;
  size_t alone_min_keys = (size_t)1 << 16;  // requests at least this long run alone (device-wide)
};

struct Stats {
  uint64_t submitted = 0, completed = 0, failed = 0, cancelled = 0, batches = 0, alone = 0, keys = 0;
  std::vector<double> latency_us;  // submit (or arrival) to completion, per completed request
  std::vector<double> queue_us;    // submit (or arrival) to launch, per completed request
  size_t scratch_total = 0, scratch_peak = 0;
};

class Server {
 public:
  Server(const Config& cfg, Executor* ex) : cfg_(cfg), ex_(ex), ledger_(ex->scratch_budget()) {
    slots_.resize(ex_->num_slots());
    worker_ = std::thread([this] { loop(); });
  }

  ~Server() { shutdown(); }

  // Non-blocking: validates, applies the budget and queue bounds, queues the request.
  // arrival_ns: the request's arrival time on the steady clock (now_ns()), from which its latency
  // is measured; 0 = the time of this call.
  ap_status submit(const uint32_t* in, uint32_t* out, size_t n, int P, uint32_t* spl, unsigned flags,
                   uint64_t* ticket, uint64_t arrival_ns = 0) {
    if (!ticket) return AP_ERR_INVALID;
    if (P < 1 || n >= AP_MAX_KEYS || (n && (!in || !out))) return AP_ERR_INVALID;
    if (n && in != out) {
      const uintptr_t a0 = (uintptr_t)in, a1 = a0 + n * 4, b0 = (uintptr_t)out, b1 = b0 + n * 4;
      if (a0 < b1 && b0 < a1) return AP_ERR_INVALID;
    }
    Request* r = new Request();
    r->in = in;
    r->out = out;
    r->n = n;
    r->P = P;
    r->spl = spl;
    r->flags = flags;
    const bool alone = n >= cfg_.alone_min_keys;
    if (Ledger::round_up(ex_->scratch_bytes(*r, alone)) > ledger_.total()) {
      delete r;
      return AP_ERR_BUDGET;
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_) {
      delete r;
      return AP_ERR_CANCELLED;
    }
    if ((int)pending_.size() >= cfg_.max_queue) {
      delete r;
      return AP_ERR_QUEUE_FULL;
    }
    r->ticket = ++next_ticket_;
    const uint64_t t_now = now_ns();
    r->t_submit = (arrival_ns && arrival_ns <= t_now) ? arrival_ns : t_now;
    tickets_[r->ticket] = r;
    pending_.push_back(r);
    stats_.submitted++;
    arrivals_++;
    if (last_arrival_ns_) {  // running mean of the gaps between arrivals (weight 1/8)
      const uint64_t gap = t_now > last_arrival_ns_ ? t_now - last_arrival_ns_ : 0;
      gap_ewma_ns_ = gap_ewma_ns_ ? gap_ewma_ns_ - gap_ewma_ns_ / 8 + gap / 8 : gap;
    }
    last_arrival_ns_ = t_now;
    *ticket = r->ticket;
    cv_work_.notify_one();
    return AP_OK;
  }

  // Final status of the ticket, or AP_ERR_TIMEOUT when it is not done within timeout_us
  // (< 0: wait forever).  A ticket whose final status was returned is forgotten.
  ap_status wait(uint64_t ticket, int64_t timeout_us) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return AP_ERR_INVALID;
    Request* r = it->second;
    auto done = [&] { return r->status >= 0; };
    if (timeout_us < 0) {
      cv_done_.wait(lk, done);
    } else if (!cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
      return AP_ERR_TIMEOUT;
    }
    const ap_status st = (ap_status)r->status;
    tickets_.erase(it);
    delete r;
    return st;
  }

  ap_status poll(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return AP_ERR_INVALID;
    Request* r = it->second;
    if (r->status < 0) return AP_ERR_TIMEOUT;
    const ap_status st = (ap_status)r->status;
    tickets_.erase(it);
    delete r;
    return st;
  }

  Stats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    Stats s = stats_;
    s.scratch_total = ledger_.total();
    s.scratch_peak = ledger_.peak();
    return s;
  }

  void reset_latencies() {
    std::lock_guard<std::mutex> lk(mu_);
    stats_.latency_us.clear();
    stats_.queue_us.clear();
  }

  // Ledger state for tests: bytes reserved now, and whether the free list is consistent.
  size_t scratch_in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return ledger_.used();
  }
  bool ledger_consistent() {
    std::lock_guard<std::mutex> lk(mu_);
    return ledger_.consistent();
  }

  // Stop accepting, cancel queued requests, let in-flight work finish, join the scheduler.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (joined_) return;
      stopping_ = true;
      for (Request* r : pending_) {
        r->status = AP_ERR_CANCELLED;
        r->t_done = now_ns();
        stats_.cancelled++;
      }
      pending_.clear();
      cv_work_.notify_all();
      cv_done_.notify_all();
    }
    worker_.join();
    std::lock_guard<std::mutex> lk(mu_);
    joined_ = true;
    for (auto& kv : tickets_) delete kv.second;
    tickets_.clear();
  }

 private:
  struct Slot {
    bool busy = false;
    std::vector<Request*> reqs;
    size_t off = 0, bytes = 0;  // the slot's scratch reservation
  };

  void finish(Request* r, ap_status st, uint64_t t) {
    r->status = st;
    r->t_done = t;
    if (st == AP_OK) {
      stats_.completed++;
      stats_.keys += r->n;
      stats_.latency_us.push_back((double)(t - r->t_submit) / 1e3);
      stats_.queue_us.push_back((double)(r->t_launch - r->t_submit) / 1e3);
    } else {
      stats_.failed++;
    }
  }

  // Takes the next unit of work from the queue head (FIFO) and reserves its scratch: a long
  // request alone, or a batch of the queued requests that are not long, in arrival order, up to
  // max_batch and the largest free range of the ledger.  Long requests behind the head wait for
  // their turn; short ones may overtake them.  A long head whose scratch is not free yet waits,
  // and until it runs only requests that need no scratch are launched, so that it is not starved;
  // likewise a short request that does not fit ends its batch.
  bool form_work(std::vector<Request*>& batch, bool& alone, size_t& off, size_t& bytes) {
    batch.clear();
    off = bytes = 0;
    if (pending_.empty()) return false;
    Request* head = pending_.front();
    size_t room;
    if (head->n >= cfg_.alone_min_keys) {
      const size_t need = ex_->scratch_bytes(*head, true);
      if (ledger_.reserve(need, &off)) {
        pending_.pop_front();
        batch.push_back(head);
        alone = true;
        bytes = need;
        return true;
      }
      room = 0;
    } else {
      room = ledger_.largest_free();
    }
    alone = false;
    size_t used = 0;
    for (auto it = pending_.begin(); it != pending_.end() && (int)batch.size() < cfg_.max_batch;) {
      Request* r = *it;
      if (r->n >= cfg_.alone_min_keys) {
        ++it;
        continue;
      }
      const size_t need = Ledger::round_up(ex_->scratch_bytes(*r, false));
      if (used + need > room) break;
      used += need;
      batch.push_back(r);
      it = pending_.erase(it);
    }
    if (batch.empty()) return false;
    if (!ledger_.reserve(used, &off)) {  // cannot happen: used <= the largest free range
      for (auto it = batch.rbegin(); it != batch.rend(); ++it) pending_.push_front(*it);
      batch.clear();
      return false;
    }
    bytes = used;
    return true;
  }

  // How long the loop polls without sleeping after an event: twice the mean gap between
  // arrivals, so that at a steady rate the next request usually finds it awake, within
  // [kSpinMinNs, kSpinMaxNs], so that a quiet server sleeps.
  uint64_t spin_window_ns() const {
    return std::min(kSpinMaxNs, std::max(kSpinMinNs, 2 * gap_ewma_ns_));
  }

  void loop() {
    // While device work is in flight, or for spin_window_ns() after the last launch, completion
    // or arrival, the loop polls without sleeping (yielding the core between polls): waking a
    // sleeping thread costs tens of microseconds, as much as a short request's device time.
    // After that it waits in steps of kPollUs while work is in flight, and blocks when there is
    // none; the default 50 us timer slack of a Linux thread would stretch every such wait to
    // ~70 us, so it is cut to 1 us.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
    ex_->thread_init();
    std::vector<Request*> batch;
    std::unique_lock<std::mutex> lk(mu_);
    uint64_t last_event = now_ns();
    uint64_t seen_arrivals = arrivals_;
    while (true) {
      // completions
      bool any_busy = false;
      for (int s = 0; s < (int)slots_.size(); ++s) {
        Slot& sl = slots_[s];
        if (!sl.busy) continue;
        lk.unlock();
        const int q = ex_->query(s);
        lk.lock();
        if (q == 0) {
          any_busy = true;
          continue;
        }
        const uint64_t t = now_ns();
        last_event = t;
        for (Request* r : sl.reqs) finish(r, q > 0 ? AP_OK : AP_ERR_DEVICE, t);
        sl.reqs.clear();
        ledger_.release(sl.off, sl.bytes);
        sl.off = sl.bytes = 0;
        sl.busy = false;
        cv_done_.notify_all();
      }
      // launches on free slots
      for (int s = 0; s < (int)slots_.size(); ++s) {
        if (slots_[s].busy) continue;
        bool alone = false;
        size_t off = 0, bytes = 0;
        if (!form_work(batch, alone, off, bytes)) break;
        const uint64_t t = now_ns();
        last_event = t;
        // test hook: requests flagged for an injected fault fail on their own, without running
        for (auto it = batch.begin(); it != batch.end();) {
          if ((*it)->flags & kInjectFault) {
            finish(*it, AP_ERR_DEVICE, t);
            it = batch.erase(it);
          } else {
            ++it;
          }
        }
        if (batch.empty()) {
          ledger_.release(off, bytes);
          cv_done_.notify_all();
          --s;  // the slot is still free
          continue;
        }
        for (Request* r : batch) r->t_launch = t;
        lk.unlock();
        const ap_status st = alone ? ex_->launch_alone(s, batch[0], off, bytes) : ex_->launch_batch(s, batch, off, bytes);
        lk.lock();
        if (alone) stats_.alone++;
        else stats_.batches++;
        if (st != AP_OK) {
          ledger_.release(off, bytes);
          const uint64_t t2 = now_ns();
          for (Request* r : batch)
            if (r->status < 0) finish(r, AP_ERR_DEVICE, t2);
          cv_done_.notify_all();
          continue;
        }
        slots_[s].busy = true;
        slots_[s].reqs = batch;
        slots_[s].off = off;
        slots_[s].bytes = bytes;
        any_busy = true;
      }
      bool idle = true;
      for (auto& sl : slots_) idle = idle && !sl.busy;
      if (stopping_ && pending_.empty() && idle) break;
      if (arrivals_ != seen_arrivals) {
        seen_arrivals = arrivals_;
        last_event = now_ns();
      }
      const uint64_t spin = spin_window_ns();
      if (any_busy || !pending_.empty()) {
        if (now_ns() - last_event < spin) {
          lk.unlock();
          std::this_thread::yield();
          lk.lock();
        } else {
          // device work in flight: poll again shortly, or earlier if a request arrives
          cv_work_.wait_for(lk, std::chrono::microseconds(kPollUs));
        }
      } else if (now_ns() - last_event < spin) {
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_work_.wait(lk, [&] { return stopping_ || !pending_.empty(); });
        last_event = now_ns();
      }
    }
  }

  Config cfg_;
  Executor* ex_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Request*> pending_;
  std::unordered_map<uint64_t, Request*> tickets_;
  std::vector<Slot> slots_;
  Stats stats_;
  uint64_t next_ticket_ = 0;
  bool stopping_ = false;
  bool joined_ = false;
  Ledger ledger_;
  uint64_t arrivals_ = 0;  // requests queued so far (the loop notes new ones to keep spinning)
  uint64_t last_arrival_ns_ = 0, gap_ewma_ns_ = 0;
  static constexpr int kPollUs = 10;  // completion polling interval after the spin window
  static constexpr uint64_t kSpinMinNs = 200000, kSpinMaxNs = 2000000;  // bounds of the spin window
  std::thread worker_;
};

}  // namespace srv
}  // namespace aps
