// Autotuner: times the launch configurations of the single-buffer and the batch
// kernels on caller-provided sample inputs and keeps the fastest.
//
// Candidates are timed in interleaved rounds (every candidate once per round, in
// a rotated order), and each candidate's score is its median over the rounds, so
// a clock ramp or a slow round does not favour whichever candidate ran last.
// The results are the same under every configuration (tested); only speed varies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/utf8v.h"
#include "common.hpp"

namespace {

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t init() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Median over rounds of each candidate's time; index of the least.
template <class Run>
int time_candidates(int ncand, int rounds, int reps, hipStream_t st, Run run, std::vector<double>* med_out) {
  Timer t;
  if (t.init() != hipSuccess) return -1;
  std::vector<std::vector<double>> ms((size_t)ncand);
  for (int c = 0; c < ncand; ++c)  // warm-up pass (clocks, caches, code objects)
    if (run(c) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  for (int r = 0; r < rounds; ++r) {
    for (int i = 0; i < ncand; ++i) {
      const int c = (i + r) % ncand;
      if (hipEventRecord(t.a, st) != hipSuccess) return -1;
      for (int k = 0; k < reps; ++k)
        if (run(c) != hipSuccess) return -1;
      if (hipEventRecord(t.b, st) != hipSuccess || hipEventSynchronize(t.b) != hipSuccess) return -1;
      float v = 0.f;
      if (hipEventElapsedTime(&v, t.a, t.b) != hipSuccess) return -1;
      ms[(size_t)c].push_back(v);
    }
  }
  std::vector<double> med((size_t)ncand);
  int best = 0;
  for (int c = 0; c < ncand; ++c) {
    auto& v = ms[(size_t)c];
    std::sort(v.begin(), v.end());
    med[(size_t)c] = v[v.size() / 2];
    if (med[(size_t)c] < med[(size_t)best]) best = c;
  }
  if (med_out) *med_out = med;
  return best;
}

}  // namespace

extern "C" {

int utf8v_autotune_single(const uint8_t* const* bufs, const size_t* lens, int nbufs, int rounds,
                          utf8v_config* best, float* times_ms, int max_times) {
  if (!bufs || !lens || nbufs < 1 || rounds < 1 || !best) return UTF8V_EINVAL;
  utf8v_config base;
  utf8v_get_config(&base);
  std::vector<utf8v_config> cand;
  for (int u : {2, 4, 8})
    for (int w : {8, 12, 16, 20, 24, 32, 40})
      for (int a : {0, 1}) {
        utf8v_config c = base;
        c.unroll = u;
        c.waves_per_cu = w;
        c.ascii = a;
        cand.push_back(c);
      }
  int64_t* out = nullptr;
  if (hipMalloc(&out, sizeof(int64_t) * (size_t)nbufs) != hipSuccess) return UTF8V_ENOMEM;
  hipStream_t st = nullptr;
  std::vector<double> med;
  const int b = time_candidates(
      (int)cand.size(), rounds, 2, st,
      [&](int c) -> hipError_t {
        utf8v_set_config(&cand[(size_t)c]);
        for (int i = 0; i < nbufs; ++i)
          if (utf8v_validate_async(bufs[i], lens[i], out + i, st) != UTF8V_OK) return hipErrorUnknown;
        return hipSuccess;
      },
      &med);
  (void)hipStreamSynchronize(st);
  (void)hipFree(out);
  if (b < 0) {
    utf8v_set_config(&base);
    return UTF8V_EHIP;
  }
  utf8v_set_config(&cand[(size_t)b]);
  *best = cand[(size_t)b];
  for (int i = 0; times_ms && i < max_times && i < (int)med.size(); ++i) times_ms[i] = (float)med[(size_t)i];
  return (int)cand.size();
}

int utf8v_autotune_batch(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                         int64_t* out_first_err, int rounds, utf8v_config* best, float* times_ms, int max_times) {
  if (!data || !offsets || n < 1 || !out_flags || !out_first_err || rounds < 1 || !best) return UTF8V_EINVAL;
  utf8v_config base;
  utf8v_get_config(&base);
  std::vector<utf8v_config> cand;
  for (int w : {4, 8, 12, 16, 20, 24, 32, 48, 64})
    for (int a : {0, 1})
      for (int u : {4, 8}) {
        utf8v_config c = base;
        c.batch_waves_per_cu = w;
        c.batch_ascii = a;
        c.batch_unroll = u;
        cand.push_back(c);
      }
  hipStream_t st = nullptr;
  std::vector<double> med;
  const int b = time_candidates(
      (int)cand.size(), rounds, 3, st,
      [&](int c) -> hipError_t {
        utf8v_set_config(&cand[(size_t)c]);
        return utf8v_validate_batch_async(data, offsets, n, out_flags, out_first_err, st) == UTF8V_OK
                   ? hipSuccess
                   : hipErrorUnknown;
      },
      &med);
  (void)hipStreamSynchronize(st);
  if (b < 0) {
    utf8v_set_config(&base);
    return UTF8V_EHIP;
  }
  utf8v_set_config(&cand[(size_t)b]);
  *best = cand[(size_t)b];
  for (int i = 0; times_ms && i < max_times && i < (int)med.size(); ++i) times_ms[i] = (float)med[(size_t)i];
  return (int)cand.size();
}

}  // extern "C"
