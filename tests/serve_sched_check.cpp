// CPU check of the serving scheduler (csrc/serve_core.hpp) with a fake backend, built
// with ThreadSanitizer by tests/test_serve_core.py.  Several client threads submit
// requests and wait for some of them; the fake backend completes batches after a
// random number of polls (out of launch order), refuses launches now and then (ring or
// staging full), and writes each request's results when its batch completes.  Checked:
// batches respect the limits and take tickets in order, at most max_inflight are out,
// batches retire in launch order, a request is reported done only after its batch and
// every earlier batch completed, every result is written exactly once, and no request
// slot is reused while its request is unfinished (max_pending backpressure).
#include <stdint.h>
#include <stdio.h>

#include <atomic>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "../paper_2010_03090_amd/csrc/serve_core.hpp"

using utf8v::ServeLimits;
using utf8v::ServeRequest;
using utf8v::ServeScheduler;

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);         \
      g_fail.store(1);                                                      \
    }                                                                       \
  } while (0)

struct Req {  // a client's request: its offsets array carries its identity
  int64_t offsets[2];
  uint8_t flags[1];
  int64_t errs[1];
  std::atomic<int> writes{0};
};

struct FakeBackend {
  ServeScheduler<FakeBackend>* sched = nullptr;
  ServeLimits lim;
  std::mt19937_64 rng{7};
  struct Batch {
    uint64_t first, count;
    int polls_left;
    bool completed;
  };
  std::vector<Batch> batches;       // every batch ever launched, in launch order
  std::vector<int> live;            // handles out (launch order)
  std::atomic<int64_t> completed_upto{-1};  // largest index b such that batches 0..b all completed
  uint64_t next_first = 0;
  int max_out = 0;

  int launch(uint64_t first, uint64_t count) {
    if (rng() % 7 == 0) return -1;  // resources not free yet
    CHECK(first == next_first);
    CHECK(count >= 1 && count <= (uint64_t)lim.max_batch_requests);
    uint64_t bytes = 0;
    int64_t strings = 0;
    for (uint64_t i = 0; i < count; ++i) {
      const ServeRequest& r = sched->slot(first + i);
      CHECK(r.state.load() == 1);
      CHECK(r.offsets[0] == (int64_t)(first + i) * 3 + 11);  // the slot holds this ticket's request
      bytes += (uint64_t)r.bytes;
      strings += r.n + 1;
    }
    CHECK(count == 1 || (bytes <= lim.max_batch_bytes && strings <= lim.max_batch_strings));
    next_first = first + count;
    const int h = (int)batches.size();
    batches.push_back(Batch{first, count, (int)(rng() % 40), false});
    live.push_back(h);
    if ((int)live.size() > max_out) max_out = (int)live.size();
    CHECK((int)live.size() <= lim.max_inflight);
    return h;
  }

  int query(int h) {
    CHECK(!live.empty() && live.front() == h);  // retirement asks for the oldest batch only
    // complete batches out of order: any live batch may finish at each poll
    for (int b : live) {
      Batch& bt = batches[(size_t)b];
      if (!bt.completed && (bt.polls_left == 0 || rng() % 3 == 0)) {
        if (bt.polls_left > 0) --bt.polls_left;
        if (bt.polls_left == 0) {
          for (uint64_t i = 0; i < bt.count; ++i) {
            const ServeRequest& r = sched->slot(bt.first + i);
            r.flags[0] = 1;
            r.errs[0] = (int64_t)(bt.first + i);
            reinterpret_cast<Req*>(const_cast<int64_t*>(r.offsets))->writes.fetch_add(1);
          }
          bt.completed = true;
        }
      }
    }
    return batches[(size_t)h].completed ? 1 : 0;
  }

  void release(int h) {
    CHECK(!live.empty() && live.front() == h);
    CHECK(batches[(size_t)h].completed);
    live.erase(live.begin());
    completed_upto.store(h);
  }
};

int main() {
  ServeLimits lim{1000, 50, 8, 3, 16};
  FakeBackend be;
  be.lim = lim;
  ServeScheduler<FakeBackend> sched(lim, &be);
  be.sched = &sched;
  std::thread worker([&] { sched.run(); });

  const int kThreads = 4, kPerThread = 1500;
  std::vector<Req> reqs((size_t)kThreads * kPerThread);
  std::vector<uint64_t> ticket_of(reqs.size());
  std::mutex submit_mu;  // tickets follow submission order; the lock ties ticket to request
  std::vector<std::thread> clients;
  for (int c = 0; c < kThreads; ++c) {
    clients.emplace_back([&, c] {
      std::mt19937_64 rng(100 + c);
      uint64_t last = 0;
      for (int i = 0; i < kPerThread; ++i) {
        Req& q = reqs[(size_t)c * kPerThread + i];
        const int64_t n = (int64_t)(rng() % 20);
        const int64_t bytes = (int64_t)(rng() % 300);
        uint64_t t;
        {
          std::lock_guard<std::mutex> lk(submit_mu);
          t = sched.submitted();
          q.offsets[0] = (int64_t)t * 3 + 11;
          q.offsets[1] = q.offsets[0] + bytes;
          const uint64_t got = sched.submit(reinterpret_cast<const uint8_t*>(&q), q.offsets, n, bytes, q.flags, q.errs);
          CHECK(got == t);
        }
        ticket_of[(size_t)c * kPerThread + i] = t;
        CHECK(i == 0 || t > last);
        last = t;
        CHECK(sched.submitted() - sched.retired() <= (uint64_t)lim.max_pending + kThreads);
        if (rng() % 5 == 0) {
          int64_t done = 0;
          CHECK(sched.wait(t, &done) == 1);
          CHECK(q.writes.load() == 1 && q.errs[0] == (int64_t)t && q.flags[0] == 1);
          CHECK(done > 0 && done <= utf8v::mono_ns());
        }
        if (rng() % 97 == 0) std::this_thread::sleep_for(std::chrono::microseconds(300));  // idle gaps
      }
    });
  }
  for (auto& t : clients) t.join();
  for (size_t i = 0; i < reqs.size(); ++i) {
    CHECK(sched.wait(ticket_of[i], nullptr) == 1);
    CHECK(reqs[i].writes.load() == 1);
    CHECK(reqs[i].errs[0] == (int64_t)ticket_of[i] && reqs[i].flags[0] == 1);
  }
  // an idle scheduler sleeps and still wakes up for a late request
  std::this_thread::sleep_for(std::chrono::milliseconds(30));
  Req late;
  {
    std::lock_guard<std::mutex> lk(submit_mu);
    late.offsets[0] = (int64_t)sched.submitted() * 3 + 11;
    late.offsets[1] = late.offsets[0] + 5;
    const uint64_t t = sched.submit(reinterpret_cast<const uint8_t*>(&late), late.offsets, 2, 5, late.flags, late.errs);
    CHECK(sched.wait(t, nullptr) == 1 && late.writes.load() == 1);
  }
  sched.stop();
  worker.join();
  CHECK(sched.retired() == reqs.size() + 1);
  CHECK(be.max_out >= 2);  // batches did overlap
  CHECK(sched.error() == 0);
  printf("scheduler ok: %zu requests, %lld batches, largest %lld, most out at once %d\n", reqs.size() + 1,
         (long long)sched.batches(), (long long)sched.max_batch(), be.max_out);
  return g_fail.load();
}
