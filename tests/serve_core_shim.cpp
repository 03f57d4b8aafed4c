// Test double: exposes the serving loop's host-side planner (ring allocator and
// batch layout) through a C interface, built with g++ by the CPU tests.
#include <stdint.h>

#include <vector>

#include "../paper_2010_03090_amd/csrc/serve_core.hpp"

extern "C" {

void* ring_new(uint64_t cap) { return new utf8v::ByteRing(cap); }
void ring_free(void* r) { delete static_cast<utf8v::ByteRing*>(r); }
int64_t ring_reserve(void* r, uint64_t n) { return static_cast<utf8v::ByteRing*>(r)->reserve(n); }
void ring_release(void* r) { static_cast<utf8v::ByteRing*>(r)->release_oldest(); }
uint64_t ring_used(void* r) { return static_cast<utf8v::ByteRing*>(r)->used(); }
uint64_t ring_capacity(void* r) { return static_cast<utf8v::ByteRing*>(r)->capacity(); }

// regions[6] = desc_at, data_at, offsets_at, flags_at, errs_at, total; returns strings
int64_t plan(int64_t count, const uint64_t* bytes, const int64_t* strings, const uint64_t* src, uint64_t desc_bytes,
             uint64_t* data_off, int64_t* str_off, uint64_t* data_bytes, uint64_t* regions) {
  std::vector<utf8v::PlanRequest> reqs((size_t)count);
  for (int64_t i = 0; i < count; ++i) reqs[(size_t)i] = utf8v::PlanRequest{bytes[i], strings[i], (uintptr_t)src[i]};
  const utf8v::BatchPlan p = utf8v::plan_batch(reqs, 0, (size_t)count, desc_bytes);
  for (int64_t i = 0; i < count; ++i) {
    data_off[i] = p.data_off[(size_t)i];
    str_off[i] = p.str_off[(size_t)i];
  }
  *data_bytes = p.data_bytes;
  const uint64_t r[6] = {p.desc_at, p.data_at, p.offsets_at, p.flags_at, p.errs_at, p.total};
  for (int i = 0; i < 6; ++i) regions[i] = r[i];
  return p.strings;
}
}
