// Where the waves that a batch string spans report their part of its first detection
// (the batch kernel's cross-wave slots).  Plain C++ (constexpr, so the kernel calls it
// too), checked on the host by tests/cross_wave_check.cpp.
//
// String k runs over the waves ws < we, and slot i belongs to wave i.  Every wave of the
// string arrives once.  With at most kFanIn waves strictly inside the string, all of them
// arrive at slot ws.  With more, the waves strictly inside it (which hold no boundary, so
// no string starts in them and their own slots are free) arrive in groups of kFanIn at the
// slot of their group's first wave, and the last arrival of each group arrives once more,
// for the group, at slot ws: slot ws then counts the first wave, the last wave and one
// arrival per group.  Atomics on one word run one after another across the device, so
// this keeps a string across thousands of waves from holding up the end of the kernel.
#pragma once

namespace utf8v {

constexpr int kFanIn = 64;

struct ArrivalPlan {
  int slot;        // the slot wave w arrives at
  int expect;      // arrivals that slot receives in all
  int top_expect;  // arrivals slot ws receives in all
};

constexpr ArrivalPlan arrival_plan(int ws, int we, int w) {
  const int inner = we - ws - 1;  // waves strictly inside the string
  const int top = inner > kFanIn ? 2 + (inner + kFanIn - 1) / kFanIn : we - ws + 1;
  ArrivalPlan p{ws, top, top};
  if (inner > kFanIn && w > ws && w < we) {
    p.slot = ws + 1 + (w - ws - 1) / kFanIn * kFanIn;
    p.expect = we - p.slot < kFanIn ? we - p.slot : kFanIn;
  }
  return p;
}

}  // namespace utf8v
