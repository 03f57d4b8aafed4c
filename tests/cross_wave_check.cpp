// Host check of the batch kernel's cross-wave arrival plan (csrc/cross_wave_plan.hpp),
// built with g++ by tests/test_serve_core.py: for strings over every span of waves up to
// a few thousand, each wave arrives once, every group slot lies strictly inside the
// string (a slot no other string uses) and receives exactly the arrivals its members
// expect, and the string's own slot receives its direct arrivals plus one per group.
#include <stdio.h>

#include <map>

#include "../paper_2010_03090_amd/csrc/cross_wave_plan.hpp"

using utf8v::arrival_plan;
using utf8v::kFanIn;

static_assert(arrival_plan(0, 1, 0).expect == 2 && arrival_plan(0, 1, 1).slot == 0, "two waves");
static_assert(arrival_plan(5, 5 + kFanIn + 2, 6).slot == 6 && arrival_plan(5, 5 + kFanIn + 2, 6).expect == kFanIn,
              "the first group");

int main() {
  int fails = 0;
  for (int ws = 0; ws < 3; ++ws)
    for (int span = 1; span < 5000; ++span) {
      const int we = ws + span;
      std::map<int, int> count;
      std::map<int, int> expect;
      const int top = arrival_plan(ws, we, ws).top_expect;
      for (int w = ws; w <= we; ++w) {
        const auto p = arrival_plan(ws, we, w);
        if (p.top_expect != top) ++fails;
        if (expect.count(p.slot) && expect[p.slot] != p.expect) ++fails;
        expect[p.slot] = p.expect;
        ++count[p.slot];
      }
      int groups = 0;
      for (const auto& kv : count) {
        if (kv.first == ws) continue;
        ++groups;
        if (!(kv.first > ws && kv.first < we) || kv.second != expect[kv.first]) ++fails;
      }
      if (count[ws] + groups != top || expect[ws] != top) ++fails;
      if (span > kFanIn + 1 && count[ws] != 2) ++fails;  // grouped: only the first and last wave arrive directly
      if (fails) {
        printf("arrival plan wrong for ws %d we %d\n", ws, we);
        return 1;
      }
    }
  printf("arrival plan ok\n");
  return 0;
}
