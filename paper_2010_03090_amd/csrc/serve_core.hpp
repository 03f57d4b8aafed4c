// Host-side planning of the serving loop: the device ring's byte allocator and the
// layout of one continuous batch.  Plain C++ (no HIP), so the same code is
// exercised by the CPU tests.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <deque>
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

}  // namespace utf8v
