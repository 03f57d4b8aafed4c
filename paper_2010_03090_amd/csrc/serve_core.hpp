// Host side of the serving loop: the device ring's byte allocator, the layout of one
// continuous batch, and the scheduler that admits requests into batches and retires
// them in order.  Plain C++ (no HIP): the server plugs in a GPU backend, the CPU tests a
// fake one (built with ThreadSanitizer).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace utf8v {

constexpr uint64_t kRingAlign = 256;

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// First-in first-out allocator over [0, cap) bytes: each reservation is one
// contiguous, kRingAlign-aligned range; reservations are released in the order they
// were made.  A reservation that does not fit before the end wraps to offset 0 and
// the skipped tail stays occupied until that reservation is released.
class ByteRing {
 public:
  explicit ByteRing(uint64_t cap) : cap_(cap / kRingAlign * kRingAlign) {}

  uint64_t capacity() const { return cap_; }
  uint64_t used() const { return used_; }
  size_t live() const { return live_.size(); }

  // Offset of a new reservation of n bytes, or -1 if it does not fit now.
  int64_t reserve(uint64_t n) {
    n = align_up(n ? n : 1, kRingAlign);
    if (n > cap_) return -1;
    uint64_t at = head_, skip = 0;
    if (live_.empty()) {
      at = 0;
      head_ = tail_ = 0;
    } else if (head_ == tail_) {  // wrapped all the way round: full
      return -1;
    } else if (head_ > tail_) {  // free space is [head, cap) and [0, tail)
      if (cap_ - head_ < n) {
        if (tail_ < n) return -1;
        skip = cap_ - head_;
        at = 0;
      }
    } else {  // free space is [head, tail)
      if (tail_ - head_ < n) return -1;
    }
    live_.push_back(Span{at, n, skip});
    used_ += n + skip;
    head_ = at + n;
    return (int64_t)at;
  }

  // Release the oldest reservation.
  void release_oldest() {
    if (live_.empty()) return;
    const Span s = live_.front();
    live_.pop_front();
    used_ -= s.size + s.skip;
    if (live_.empty()) {
      head_ = tail_ = 0;
    } else {
      tail_ = live_.front().at;
    }
  }

 private:
  struct Span {
    uint64_t at, size, skip;  // skip: bytes left unused at the end of the ring before `at`
  };
  uint64_t cap_, head_ = 0, tail_ = 0, used_ = 0;
  std::deque<Span> live_;
};

// One request as the planner sees it.
struct PlanRequest {
  uint64_t bytes;   // payload bytes
  int64_t strings;  // strings in the request
  uintptr_t src;    // address of its payload (the device copy keeps the same alignment mod 16)
};

// Layout of a continuous batch inside one ring reservation: the descriptor table,
// the payloads (request r at data_off[r], aligned like its source mod 16, with a
// padding string after it so requests stay contiguous in the CSR form), the
// rebased offsets, and the per-string results.
struct BatchPlan {
  std::vector<uint64_t> data_off;  // per request, relative to the data region
  std::vector<int64_t> str_off;    // per request, index of its first string in the batch
  int64_t strings = 0;             // strings in the batch, padding strings included
  uint64_t data_bytes = 0;         // end of the last payload
  // region offsets inside the reservation
  uint64_t desc_at = 0, data_at = 0, offsets_at = 0, flags_at = 0, errs_at = 0, total = 0;
};

// Lay out requests[first, first+count) as one batch; desc_bytes is the size of one
// descriptor.  The ring and every region offset are kRingAlign-aligned, so a payload
// at data_off has the device address alignment of data_off.
inline BatchPlan plan_batch(const std::vector<PlanRequest>& reqs, size_t first, size_t count, uint64_t desc_bytes) {
  BatchPlan p;
  p.data_off.resize(count);
  p.str_off.resize(count);
  uint64_t pos = 0;
  int64_t s = 0;
  for (size_t i = 0; i < count; ++i) {
    const PlanRequest& r = reqs[first + i];
    // same address modulo 16 as the source, so both copy sides use aligned 16-byte words
    uint64_t at = (pos & ~uint64_t(15)) + (r.src & 15u);
    if (at < pos) at += 16;
    pos = at;
    p.data_off[i] = pos;
    p.str_off[i] = s;
    pos += r.bytes;
    s += r.strings + (i + 1 < count ? 1 : 0);  // padding string between requests
  }
  p.strings = s;
  p.data_bytes = pos;
  p.desc_at = 0;
  p.data_at = align_up(desc_bytes * count, kRingAlign);
  p.offsets_at = align_up(p.data_at + p.data_bytes + 16, kRingAlign);
  p.flags_at = align_up(p.offsets_at + 8 * (uint64_t)(s + 1), kRingAlign);
  p.errs_at = align_up(p.flags_at + (uint64_t)s, kRingAlign);
  p.total = align_up(p.errs_at + 8 * (uint64_t)s, kRingAlign);
  return p;
}

inline int64_t mono_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// One submitted request: a CSR batch of strings (offsets[0..n], payload bytes) and the
// arrays its results go to.
// The fields other than the atomics are written by submit before it publishes the state
// and read by the scheduler thread after it sees the state published.
struct ServeRequest {
  const uint8_t* data = nullptr;
  const int64_t* offsets = nullptr;
  int64_t n = 0, bytes = 0;
  uint8_t* flags = nullptr;
  int64_t* errs = nullptr;
  int64_t submit_ns = 0;
  std::atomic<uint64_t> ticket{~uint64_t(0)};  // the request the slot holds
  std::atomic<int64_t> done_ns{0};             // when the scheduler saw it done
  std::atomic<int> state{0};                   // 0 free, 1 submitted, 2 in a batch, 3 done
};

struct ServeLimits {
  uint64_t max_batch_bytes;   // payload bytes per batch (a single larger request is refused at submit)
  int64_t max_batch_strings;  // strings per batch, one separator string per request included
  int max_batch_requests;     // requests per batch
  int max_inflight;           // batches launched and not yet retired
  int max_pending;            // submitted and not yet retired requests (size of the request table)
};

// Continuous batching.  Clients submit requests from any thread and get tickets in
// submission order; one scheduler thread (run) admits submitted requests in ticket
// order into a batch, up to the limits, whenever fewer than max_inflight batches are
// out, hands the batch to the backend, and retires batches in launch order once the
// backend reports them done.  The backend is called from the scheduler thread only:
//   int  launch(uint64_t first, uint64_t count)  handle >= 0; -1 if its resources are
//                                                not free yet (nothing started)
//   int  query(int handle)                       1 done, 0 still running, < 0 failed
//   void release(int handle)                     in launch order, after query said done
// With nothing submitted and nothing out, the scheduler sleeps until a submit or stop.
template <class Backend>
class ServeScheduler {
 public:
  ServeScheduler(const ServeLimits& lim, Backend* be)
      : lim_(lim), be_(be), slots_(new ServeRequest[(size_t)lim.max_pending]) {}

  ServeRequest& slot(uint64_t t) { return slots_[t % (uint64_t)lim_.max_pending]; }
  const ServeLimits& limits() const { return lim_; }

  // Client side.  Blocks while max_pending requests are unfinished.
  uint64_t submit(const uint8_t* data, const int64_t* offsets, int64_t n, int64_t bytes, uint8_t* flags,
                  int64_t* errs) {
    const uint64_t t = next_ticket_.fetch_add(1);
    while (t - retired_.load(std::memory_order_acquire) >= (uint64_t)lim_.max_pending) std::this_thread::yield();
    ServeRequest& r = slot(t);
    r.ticket.store(t);
    r.done_ns.store(0);
    r.data = data;
    r.offsets = offsets;
    r.n = n;
    r.bytes = bytes;
    r.flags = flags;
    r.errs = errs;
    r.submit_ns = mono_ns();
    r.state.store(1, std::memory_order_release);
    if (sleeping_.load()) {
      std::lock_guard<std::mutex> lk(mu_);
      cv_.notify_one();
    }
    return t;
  }

  // 1 if the request is done (its results are in place), 0 if not yet, the server's
  // error status (< 0) if it failed.  *done_ns: when the scheduler saw it done; once its
  // slot holds a later request (max_pending requests were submitted after it), the time
  // of this call, which is later.
  int poll(uint64_t ticket, int64_t* done_ns) {
    if (ticket >= retired_.load(std::memory_order_acquire)) return error_.load();
    if (done_ns) {
      const ServeRequest& r = slot(ticket);
      int64_t d = r.done_ns.load(std::memory_order_acquire);
      if (r.ticket.load(std::memory_order_acquire) != ticket || d == 0) d = mono_ns();
      *done_ns = d;
    }
    return 1;
  }

  int wait(uint64_t ticket, int64_t* done_ns) {
    for (;;) {
      const int r = poll(ticket, done_ns);
      if (r != 0) return r;
      std::this_thread::yield();
    }
  }

  uint64_t submitted() const { return next_ticket_.load(); }
  uint64_t retired() const { return retired_.load(); }
  int64_t batches() const { return batches_.load(); }
  int64_t max_batch() const { return max_batch_.load(); }
  int error() const { return error_.load(); }
  void set_error(int e) {
    int z = 0;
    error_.compare_exchange_strong(z, e);
  }

  void stop() {
    stop_.store(true);
    std::lock_guard<std::mutex> lk(mu_);
    cv_.notify_one();
  }

  // The scheduler thread: until stop() and everything submitted is done.
  void run() {
    for (;;) {
      bool progress = retire_ready();
      if ((int)inflight_.size() < lim_.max_inflight) progress = admit() || progress;
      const bool none_waiting = sched_ >= next_ticket_.load();
      if (stop_.load() && inflight_.empty() && none_waiting) break;
      if (progress) continue;
      if (inflight_.empty() && none_waiting) {
        std::unique_lock<std::mutex> lk(mu_);
        sleeping_.store(true);
        if (sched_ >= next_ticket_.load() && !stop_.load())
          cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(5));
        sleeping_.store(false);
      } else {
        std::this_thread::yield();
      }
    }
  }

 private:
  struct InFlight {
    uint64_t first, count;
    int handle;
  };

  bool retire_ready() {
    bool any = false;
    while (!inflight_.empty()) {
      const InFlight f = inflight_.front();
      const int q = be_->query(f.handle);
      if (q == 0) break;
      if (q < 0) set_error(q);
      const int64_t t = mono_ns();
      for (uint64_t i = 0; i < f.count; ++i) {
        ServeRequest& r = slot(f.first + i);
        r.done_ns.store(t, std::memory_order_release);
        r.state.store(3, std::memory_order_release);
      }
      be_->release(f.handle);
      inflight_.pop_front();
      retired_.store(f.first + f.count, std::memory_order_release);
      any = true;
    }
    return any;
  }

  // Admit submitted requests in ticket order up to the batch limits and launch them.
  bool admit() {
    uint64_t count = 0, bytes = 0;
    int64_t strings = 0;
    const uint64_t avail = next_ticket_.load(std::memory_order_acquire);
    while (count < (uint64_t)lim_.max_batch_requests && sched_ + count < avail) {
      const ServeRequest& r = slot(sched_ + count);
      if (r.state.load(std::memory_order_acquire) != 1) break;  // ticket taken, request not yet written
      if (count > 0 && (bytes + (uint64_t)r.bytes > lim_.max_batch_bytes ||
                        strings + r.n + 1 > lim_.max_batch_strings))
        break;
      bytes += (uint64_t)r.bytes;
      strings += r.n + 1;
      ++count;
    }
    if (count == 0) return false;
    const int h = be_->launch(sched_, count);
    if (h < 0) return false;
    for (uint64_t i = 0; i < count; ++i) slot(sched_ + i).state.store(2, std::memory_order_relaxed);
    inflight_.push_back(InFlight{sched_, count, h});
    sched_ += count;
    batches_.fetch_add(1);
    if ((int64_t)count > max_batch_.load()) max_batch_.store((int64_t)count);
    return true;
  }

  ServeLimits lim_;
  Backend* be_;
  std::unique_ptr<ServeRequest[]> slots_;
  std::atomic<uint64_t> next_ticket_{0};
  std::atomic<uint64_t> retired_{0};  // tickets below this are done
  uint64_t sched_ = 0;                // next ticket to admit (scheduler thread only)
  std::deque<InFlight> inflight_;     // scheduler thread only
  std::atomic<bool> stop_{false}, sleeping_{false};
  std::atomic<int> error_{0};
  std::atomic<int64_t> batches_{0}, max_batch_{0};
  std::mutex mu_;
  std::condition_variable cv_;
};

}  // namespace utf8v
