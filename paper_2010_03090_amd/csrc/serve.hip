// Serving loop: continuous batching of validation requests on one GPU.
//
// Clients submit requests (a CSR batch of strings in pinned host memory) at any
// time.  One scheduler thread admits pending requests, in arrival order, into a
// device ring of a fixed byte budget, and launches them as one batch as soon as a
// batch slot is free, so requests that arrive while others are on the GPU join
// the next batch and batches overlap on alternating streams.  Per batch, on its
// stream:
//   1. the descriptor table (and its lookup tables) is copied to the ring, or, for a
//      small batch, passed in the kernel arguments;
//   2. serve_gather reads the payloads and offsets straight from pinned host
//      memory into the ring, rebasing the offsets so the requests form one CSR
//      batch (a padding string separates consecutive requests);
//   3. the batch validator (one launch) runs over it;
//   4. serve_scatter writes each request's flags and first-error offsets back
//      into its pinned host result arrays (a batch of one request has the
//      validator write them there itself);
//   5. an event marks the batch; the scheduler retires batches in order, stamps
//      their requests done and releases their ring space.
// A string's result depends only on its own bytes (each string is its own
// stream), so a request's results are the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <chrono>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "../../include/utf8v.h"
#include "common.hpp"
#include "serve_core.hpp"

namespace utf8v {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One request of a batch as the gather / scatter kernels see it.
struct ServeDesc {
  const uint8_t* src;      // payload: bytes [0, bytes) (device-accessible host memory)
  const int64_t* src_off;  // its n+1 offsets; src_off[0] is the payload start
  uint8_t* dst_flags;      // n results
  int64_t* dst_err;
  int64_t n;
  int64_t bytes;
  int64_t data_off;  // payload start in the batch data region
  int64_t str_off;   // index of its first string in the batch
};

constexpr int kGatherChunk = 4096;  // payload bytes per gather workgroup (16 per thread)
constexpr int kStringBlock = 256;   // strings per offsets / scatter workgroup

// The batch's descriptor table and its two lookup tables: chunk_req[c] / block_req[b]
// name the first request overlapping payload chunk c / string block b.  Either in the
// ring (copied before the gather) or, for small batches, in the kernel arguments.
struct RingTables {
  const ServeDesc* d;
  const int32_t* chunk_req;
  const int32_t* block_req;
  __device__ __forceinline__ const ServeDesc& desc(int r) const { return d[r]; }
  __device__ __forceinline__ int chunk(int64_t c) const { return chunk_req[c]; }
  __device__ __forceinline__ int block(int64_t b) const { return block_req[b]; }
};

constexpr int kInlineReqs = 16;      // small-batch limits: the tables fit the kernel arguments
constexpr int kInlineChunks = 320;
constexpr int kInlineBlocks = 384;

struct InlineTables {
  ServeDesc d[kInlineReqs];
  int32_t chunk_req[kInlineChunks];
  int32_t block_req[kInlineBlocks];
  __device__ __forceinline__ const ServeDesc& desc(int r) const { return d[r]; }
  __device__ __forceinline__ int chunk(int64_t c) const { return chunk_req[c]; }
  __device__ __forceinline__ int block(int64_t b) const { return block_req[b]; }
};

// Payload chunks first, then offset blocks.
template <class T>
__global__ __launch_bounds__(256) void serve_gather(T t, int nreq, int64_t chunks, uint8_t* __restrict__ data,
                                                    int64_t data_end, int64_t* __restrict__ offs, int64_t strings) {
  const int64_t b = blockIdx.x;
  if (b < chunks) {
    const int64_t p = b * kGatherChunk + threadIdx.x * 16;  // this thread's 16-byte word of the data region
    if (p >= data_end) return;
    for (int r = t.chunk(b); r < nreq && t.desc(r).data_off < p + 16; ++r) {
      const ServeDesc& d = t.desc(r);
      const int64_t s0 = d.data_off, s1 = s0 + d.bytes;
      if (s1 <= p) continue;
      if (s0 <= p && p + 16 <= s1) {  // whole word inside the payload: same alignment on both sides
        *reinterpret_cast<u32x4*>(data + p) = *reinterpret_cast<const u32x4*>(d.src + (p - s0));
      } else {
        const int64_t a = p > s0 ? p : s0, e = p + 16 < s1 ? p + 16 : s1;
        for (int64_t q = a; q < e; ++q) data[q] = d.src[q - s0];
      }
    }
    return;
  }
  const int64_t e = (b - chunks) * kStringBlock + threadIdx.x;  // boundary index
  if (e > strings) return;
  if (e == strings) {  // end of the last payload
    offs[e] = t.desc(nreq - 1).data_off + t.desc(nreq - 1).bytes;
    return;
  }
  int r = t.block(b - chunks);
  while (r + 1 < nreq && t.desc(r + 1).str_off <= e) ++r;
  const ServeDesc& d = t.desc(r);
  const int64_t k = e - d.str_off;  // k <= n: boundary k of request r (k == n: its padding string)
  offs[e] = k < d.n ? d.data_off + (d.src_off[k] - d.src_off[0]) : d.data_off + d.bytes;
}

template <class T>
__global__ __launch_bounds__(256) void serve_scatter(T t, int nreq, const uint8_t* __restrict__ flags,
                                                     const int64_t* __restrict__ errs, int64_t strings) {
  const int64_t e = (int64_t)blockIdx.x * kStringBlock + threadIdx.x;
  if (e >= strings) return;
  int r = t.block(blockIdx.x);
  while (r + 1 < nreq && t.desc(r + 1).str_off <= e) ++r;
  const ServeDesc& d = t.desc(r);
  const int64_t k = e - d.str_off;
  if (k < d.n) {
    d.dst_flags[k] = flags[e];
    d.dst_err[k] = errs[e];
  }
}

}  // namespace utf8v

namespace {

using namespace utf8v;

int64_t now_ns() { return mono_ns(); }

struct Staging {  // pinned host image of one batch's descriptor region
  uint8_t* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool busy = false;
};

struct GpuBackend;

}  // namespace

struct utf8v_server {
  utf8v_server_config cfg;
  int dev = 0, cus = 1;
  std::vector<hipStream_t> streams;
  std::vector<unsigned long long*> wave_slots;  // per stream: cross-wave slots of the batch kernel
  uint8_t* ring = nullptr;
  ByteRing alloc{0};
  std::vector<Staging> staging;
  int next_stream = 0;
  std::unique_ptr<GpuBackend> backend;
  std::unique_ptr<ServeScheduler<GpuBackend>> sched;
  std::thread worker;
};

namespace {

// The scheduler's backend: one batch = one ring reservation + one staging buffer, four
// steps on the next stream, and an event that marks the batch done.
struct GpuBackend {
  utf8v_server* s;
  int launch(uint64_t first, uint64_t count);
  int query(int h) {
    const hipError_t q = hipEventQuery(s->staging[(size_t)h].ev);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
      (void)hipGetLastError();
      return UTF8V_EHIP;
    }
    return 1;
  }
  void release(int h) {
    s->staging[(size_t)h].busy = false;
    s->alloc.release_oldest();
  }
};

// Table sizes in the descriptor region of a batch.
size_t desc_region_bytes(size_t nreq, uint64_t data_bytes, int64_t strings) {
  const size_t chunks = (size_t)((data_bytes + kGatherChunk - 1) / kGatherChunk) + 1;
  const size_t blocks = (size_t)((strings + 1 + kStringBlock - 1) / kStringBlock) + 1;
  return align_up(sizeof(ServeDesc) * nreq, 256) + align_up(4 * chunks, 256) + align_up(4 * blocks, 256);
}

// Ring bytes of the largest batch the limits allow.
uint64_t max_footprint(const utf8v_server_config& c) {
  const uint64_t r = (uint64_t)c.max_batch_requests, sn = (uint64_t)c.max_batch_strings + r;
  const uint64_t data = c.max_batch_bytes + 16 * r;
  return align_up(desc_region_bytes((size_t)r, data, (int64_t)sn), kRingAlign) + align_up(data + 16, kRingAlign) +
         align_up(8 * (sn + 1), kRingAlign) + align_up(sn, kRingAlign) + align_up(8 * sn, kRingAlign);
}

// Plan, stage and enqueue tickets [first, first+count) as one batch; the staging index
// is the batch's handle.  -1 if the ring or a staging buffer is not free yet (nothing is
// enqueued then).
int GpuBackend::launch(uint64_t first, uint64_t count) {
  auto& staging = s->staging;
  auto& alloc = s->alloc;
  auto slot = [this](uint64_t t) -> const ServeRequest& { return s->sched->slot(t); };
  int si = -1;
  for (size_t i = 0; i < staging.size(); ++i)
    if (!staging[i].busy) { si = (int)i; break; }
  if (si < 0) return -1;
  std::vector<PlanRequest> reqs(count);
  for (uint64_t i = 0; i < count; ++i) {
    const ServeRequest& r = slot(first + i);
    reqs[i] = PlanRequest{(uint64_t)r.bytes, r.n, reinterpret_cast<uintptr_t>(r.data + r.offsets[0])};
  }
  BatchPlan plan = plan_batch(reqs, 0, count, sizeof(ServeDesc));
  const size_t dbytes = desc_region_bytes(count, plan.data_bytes, plan.strings);
  // the descriptor region replaces the plan's descriptor table
  const uint64_t shift = align_up(dbytes, kRingAlign) - plan.data_at;
  plan.data_at += shift; plan.offsets_at += shift; plan.flags_at += shift; plan.errs_at += shift; plan.total += shift;
  Staging& stg = staging[si];
  if (dbytes > stg.cap) {
    s->sched->set_error(UTF8V_ENOMEM);
    return -1;
  }
  const int64_t at = alloc.reserve(plan.total);
  if (at < 0) return -1;
  uint8_t* base = s->ring + at;
  // descriptor region image
  ServeDesc* desc = reinterpret_cast<ServeDesc*>(stg.host);
  const size_t chunks = (size_t)((plan.data_bytes + kGatherChunk - 1) / kGatherChunk);
  const size_t blocks = (size_t)((plan.strings + 1 + kStringBlock - 1) / kStringBlock);
  int32_t* chunk_req = reinterpret_cast<int32_t*>(stg.host + align_up(sizeof(ServeDesc) * count, 256));
  int32_t* block_req = reinterpret_cast<int32_t*>(reinterpret_cast<uint8_t*>(chunk_req) +
                                                  align_up(4 * (chunks + 1), 256));
  for (uint64_t i = 0; i < count; ++i) {
    const ServeRequest& r = slot(first + i);
    desc[i] = ServeDesc{r.data + r.offsets[0], r.offsets, r.flags, r.errs, r.n, r.bytes,
                        (int64_t)plan.data_off[i], plan.str_off[i]};
  }
  {  // first request overlapping each payload chunk / string block
    size_t r = 0;
    for (size_t c = 0; c < chunks; ++c) {
      const uint64_t lo = (uint64_t)c * kGatherChunk;
      while (r + 1 < count && plan.data_off[r] + reqs[r].bytes <= lo) ++r;
      chunk_req[c] = (int32_t)r;
    }
    r = 0;
    for (size_t b = 0; b < blocks; ++b) {
      const int64_t lo = (int64_t)b * kStringBlock;
      while (r + 1 < count && plan.str_off[r + 1] <= lo) ++r;
      block_req[b] = (int32_t)r;
    }
  }
  hipStream_t st = s->streams[(size_t)s->next_stream];
  unsigned long long* wslots = s->wave_slots[(size_t)s->next_stream];
  s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
  const ServeDesc* ddesc = reinterpret_cast<const ServeDesc*>(base);
  const int32_t* dchunk = reinterpret_cast<const int32_t*>(base + (reinterpret_cast<uint8_t*>(chunk_req) - stg.host));
  const int32_t* dblock = reinterpret_cast<const int32_t*>(base + (reinterpret_cast<uint8_t*>(block_req) - stg.host));
  uint8_t* data = base + plan.data_at;
  int64_t* offs = reinterpret_cast<int64_t*>(base + plan.offsets_at);
  uint8_t* flags = base + plan.flags_at;
  int64_t* errs = reinterpret_cast<int64_t*>(base + plan.errs_at);
  const size_t used = (reinterpret_cast<uint8_t*>(block_req) - stg.host) + 4 * blocks;
  const int64_t grid = (int64_t)chunks + (int64_t)blocks;
  const int64_t sblocks = (plan.strings + kStringBlock - 1) / kStringBlock;
  // small batches carry the tables in the kernel arguments: no copy ahead of the gather
  const bool inline_tables = count <= (uint64_t)kInlineReqs && chunks <= (size_t)kInlineChunks &&
                             blocks <= (size_t)kInlineBlocks;
  InlineTables it;
  hipError_t e = hipSuccess;
  if (inline_tables) {
    memcpy(it.d, desc, sizeof(ServeDesc) * count);
    memcpy(it.chunk_req, chunk_req, 4 * chunks);
    memcpy(it.block_req, block_req, 4 * blocks);
    hipLaunchKernelGGL(serve_gather<InlineTables>, dim3((unsigned)grid), dim3(256), 0, st, it, (int)count,
                       (int64_t)chunks, data, (int64_t)plan.data_bytes, offs, plan.strings);
    e = hipGetLastError();
  } else {
    e = hipMemcpyAsync(base, stg.host, used, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(serve_gather<RingTables>, dim3((unsigned)grid), dim3(256), 0, st,
                         RingTables{ddesc, dchunk, dblock}, (int)count, (int64_t)chunks, data,
                         (int64_t)plan.data_bytes, offs, plan.strings);
      e = hipGetLastError();
    }
  }
  // A batch of one request (strings = the request's strings, in order) writes its results
  // straight into the request's pinned host arrays: no scatter step after it.
  const bool direct = count == 1;
  if (e == hipSuccess) {
    TuneBatch tb;
    utf8v_config c;
    utf8v_get_config(&c);
    tb.waves_per_cu = c.batch_waves_per_cu;
    tb.ascii = c.batch_ascii;
    tb.unroll = c.batch_unroll;
    const ServeRequest& r0 = slot(first);
    e = utf8v::launch_batch(batch_args(data, offs, plan.strings, direct ? r0.flags : flags,
                                       direct ? r0.errs : errs, wslots),
                            tb, s->cus, st);
  }
  if (e == hipSuccess && sblocks > 0 && !direct) {
    if (inline_tables)
      hipLaunchKernelGGL(serve_scatter<InlineTables>, dim3((unsigned)sblocks), dim3(256), 0, st, it, (int)count,
                         flags, errs, plan.strings);
    else
      hipLaunchKernelGGL(serve_scatter<RingTables>, dim3((unsigned)sblocks), dim3(256), 0, st,
                         RingTables{ddesc, dchunk, dblock}, (int)count, flags, errs, plan.strings);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(stg.ev, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    s->sched->set_error(UTF8V_EHIP);
    // nothing more runs on this server; the batch is retired when its event reports
  }
  stg.busy = true;
  return si;
}

thread_local int g_serve_status = UTF8V_OK;

int fail(int s) { g_serve_status = s; return s; }

bool device_accessible(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type != hipMemoryTypeUnregistered;
}

bool host_readable(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost || attr.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" {

int utf8v_server_default_config(utf8v_server_config* cfg) {
  if (!cfg) return UTF8V_EINVAL;
  cfg->budget_bytes = 8ull << 30;
  cfg->max_batch_bytes = 64ull << 20;
  cfg->max_batch_strings = 4ll << 20;
  cfg->max_batch_requests = 4096;
  cfg->max_inflight = 4;
  cfg->streams = 2;
  cfg->max_pending = 1 << 18;
  return UTF8V_OK;
}

int utf8v_server_create(const utf8v_server_config* cfg, utf8v_server** out) {
  if (!cfg || !out) return UTF8V_EINVAL;
  if (cfg->max_batch_bytes == 0 || cfg->max_batch_strings < 1 || cfg->max_batch_strings > kMaxBatchStrings / 2 ||
      cfg->max_batch_requests < 1 ||
      cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->streams < 1 || cfg->streams > 8 ||
      cfg->max_pending < 1 || cfg->budget_bytes < max_footprint(*cfg))
    return UTF8V_EINVAL;
  std::unique_ptr<utf8v_server> s(new utf8v_server);
  s->cfg = *cfg;
  hipError_t e = hipGetDevice(&s->dev);
  if (e != hipSuccess) return UTF8V_EHIP;
  s->cus = utf8v_num_cus() > 0 ? utf8v_num_cus() : 1;
  s->alloc = ByteRing(cfg->budget_bytes);
  s->backend.reset(new GpuBackend{s.get()});
  s->sched.reset(new ServeScheduler<GpuBackend>(
      ServeLimits{cfg->max_batch_bytes, cfg->max_batch_strings, cfg->max_batch_requests, cfg->max_inflight,
                  cfg->max_pending},
      s->backend.get()));
  e = hipMalloc(&s->ring, s->alloc.capacity());
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? UTF8V_ENOMEM : UTF8V_EHIP;
  const size_t scap = desc_region_bytes((size_t)cfg->max_batch_requests,
                                        cfg->max_batch_bytes + 16ull * (uint64_t)cfg->max_batch_requests,
                                        cfg->max_batch_strings + cfg->max_batch_requests);
  s->staging.resize((size_t)cfg->max_inflight);
  for (auto& st : s->staging) {
    e = hipHostMalloc(&st.host, scap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming);
    if (e != hipSuccess) break;
    st.cap = scap;
  }
  for (int i = 0; e == hipSuccess && i < cfg->streams; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    s->streams.push_back(st);
    unsigned long long* ws = nullptr;
    const int n = s->cus * 64;  // one word per possible wave of the batch grid
    e = hipMalloc(&ws, sizeof(unsigned long long) * n);
    if (e != hipSuccess) break;
    s->wave_slots.push_back(ws);
    e = utf8v::launch_batch_slots_init(ws, n, st);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    utf8v_server_destroy(s.release());
    return UTF8V_EHIP;
  }
  utf8v_server* raw = s.release();
  raw->worker = std::thread([raw] {
    (void)hipSetDevice(raw->dev);
    raw->sched->run();
  });
  *out = raw;
  return UTF8V_OK;
}

int utf8v_server_submit(utf8v_server* s, const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                        int64_t* out_first_err, uint64_t* ticket) {
  if (!s || !offsets || n < 0 || !ticket) return fail(UTF8V_EINVAL);
  if (n > 0 && (!out_flags || !out_first_err)) return fail(UTF8V_EINVAL);
  if (!host_readable(offsets)) return fail(UTF8V_ENOTDEVICE);
  const int64_t bytes = offsets[n] - offsets[0];
  if (offsets[0] < 0 || bytes < 0) return fail(UTF8V_EINVAL);
  if (bytes > 0 && !data) return fail(UTF8V_EINVAL);
  if ((bytes > 0 && !device_accessible(data)) || (n > 0 && (!device_accessible(out_flags) ||
                                                             !device_accessible(out_first_err))))
    return fail(UTF8V_ENOTDEVICE);
  if ((uint64_t)bytes > s->cfg.max_batch_bytes || n + 1 > s->cfg.max_batch_strings) return fail(UTF8V_EINVAL);
  if (s->sched->error()) return fail(s->sched->error());
  *ticket = s->sched->submit(data, offsets, n, bytes, out_flags, out_first_err);
  return UTF8V_OK;
}

int utf8v_server_poll(utf8v_server* s, uint64_t ticket, int64_t* done_ns) {
  if (!s) return UTF8V_EINVAL;
  return s->sched->poll(ticket, done_ns);
}

int utf8v_server_wait(utf8v_server* s, uint64_t ticket, int64_t* done_ns) {
  if (!s || ticket >= s->sched->submitted()) return UTF8V_EINVAL;
  const int r = s->sched->wait(ticket, done_ns);
  return r < 0 ? r : UTF8V_OK;
}

int utf8v_server_stats(utf8v_server* s, int64_t* out4) {
  if (!s || !out4) return UTF8V_EINVAL;
  out4[0] = (int64_t)s->sched->retired();
  out4[1] = s->sched->batches();
  out4[2] = s->sched->max_batch();
  out4[3] = (int64_t)s->alloc.capacity();
  return UTF8V_OK;
}

int utf8v_server_destroy(utf8v_server* s) {
  if (!s) return UTF8V_EINVAL;
  if (s->sched) s->sched->stop();
  if (s->worker.joinable()) s->worker.join();
  for (auto st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& st : s->staging) {
    if (st.ev) (void)hipEventDestroy(st.ev);
    if (st.host) (void)hipHostFree(st.host);
  }
  for (auto p : s->wave_slots) (void)hipFree(p);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  if (s->ring) (void)hipFree(s->ring);
  const int err = s->sched ? s->sched->error() : 0;
  delete s;
  return err;
}

int64_t utf8v_clock_ns(void) { return now_ns(); }

int utf8v_serve_replay(const utf8v_server_config* cfg, int mode, const uint8_t* const* req_data,
                       const int64_t* const* req_offsets, const int64_t* req_n, uint8_t* const* req_flags,
                       int64_t* const* req_errs, int npool, const int64_t* arrival_ns, const int32_t* pick,
                       int64_t nreq, int64_t* latency_ns, int64_t* span_ns) {
  if (!cfg || !req_data || !req_offsets || !req_n || !req_flags || !req_errs || npool < 1 || !arrival_ns || !pick ||
      nreq < 1 || !latency_ns || (mode != 0 && mode != 1))
    return UTF8V_EINVAL;
  for (int64_t i = 0; i < nreq; ++i)
    if (pick[i] < 0 || pick[i] >= npool || (i > 0 && arrival_ns[i] < arrival_ns[i - 1])) return UTF8V_EINVAL;
  auto wait_until = [](int64_t t) {
    while (now_ns() < t) {
    }
  };
  if (mode == 0) {  // continuous batching server
    utf8v_server* srv = nullptr;
    int rc = utf8v_server_create(cfg, &srv);
    if (rc) return rc;
    std::vector<uint64_t> tickets((size_t)nreq);
    std::atomic<int64_t> published{0};
    std::atomic<int> werr{0};
    const int64_t t0 = now_ns() + 2000000;
    std::thread collector([&] {
      for (int64_t i = 0; i < nreq; ++i) {
        while (published.load(std::memory_order_acquire) <= i) std::this_thread::yield();
        int64_t done = 0;
        const int r = utf8v_server_wait(srv, tickets[(size_t)i], &done);
        if (r) { werr.store(r); done = now_ns(); }
        latency_ns[i] = done - (t0 + arrival_ns[i]);
        if (span_ns && i == nreq - 1) *span_ns = done - (t0 + arrival_ns[0]);
      }
    });
    for (int64_t i = 0; i < nreq && !rc; ++i) {
      wait_until(t0 + arrival_ns[i]);
      const int k = pick[i];
      rc = utf8v_server_submit(srv, req_data[k], req_offsets[k], req_n[k], req_flags[k], req_errs[k],
                               &tickets[(size_t)i]);
      if (!rc) published.store(i + 1, std::memory_order_release);
    }
    if (rc) {  // let the collector finish on what was submitted
      const int64_t done_count = published.load();
      for (int64_t i = done_count; i < nreq; ++i) latency_ns[i] = -1;
      published.store(INT64_MAX);
    }
    collector.join();
    const int d = utf8v_server_destroy(srv);
    return rc ? rc : (werr.load() ? werr.load() : d);
  }
  // one synchronous launch per request, first come first served
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return UTF8V_EHIP;
  const int cus = utf8v_num_cus() > 0 ? utf8v_num_cus() : 1;
  int64_t max_b = 0, max_n = 0;
  for (int k = 0; k < npool; ++k) {
    max_b = std::max(max_b, req_offsets[k][req_n[k]] - req_offsets[k][0]);
    max_n = std::max(max_n, req_n[k]);
  }
  uint8_t *dd = nullptr, *df = nullptr;
  int64_t *doff = nullptr, *de = nullptr;
  unsigned long long* ws = nullptr;
  hipStream_t st = nullptr;
  hipError_t e = hipMalloc(&dd, (size_t)max_b + 16);
  if (e == hipSuccess) e = hipMalloc(&doff, 8 * (size_t)(max_n + 1));
  if (e == hipSuccess) e = hipMalloc(&df, (size_t)max_n + 1);
  if (e == hipSuccess) e = hipMalloc(&de, 8 * (size_t)max_n + 8);
  if (e == hipSuccess) e = hipMalloc(&ws, sizeof(unsigned long long) * cus * 64);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e == hipSuccess) e = utf8v::launch_batch_slots_init(ws, cus * 64, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  utf8v_config c;
  utf8v_get_config(&c);
  TuneBatch tb;
  tb.waves_per_cu = c.batch_waves_per_cu;
  tb.ascii = c.batch_ascii;
  tb.unroll = c.batch_unroll;
  const int64_t t0 = now_ns() + 2000000;
  for (int64_t i = 0; i < nreq && e == hipSuccess; ++i) {
    wait_until(t0 + arrival_ns[i]);
    const int k = pick[i];
    const int64_t n = req_n[k], o0 = req_offsets[k][0], bytes = req_offsets[k][n] - o0;
    if (bytes > 0) e = hipMemcpyAsync(dd, req_data[k] + o0, (size_t)bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(doff, req_offsets[k], 8 * (size_t)(n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && n > 0)
      e = utf8v::launch_batch(batch_args(dd - o0, doff, n, df, de, ws), tb, cus, st);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(req_flags[k], df, (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(req_errs[k], de, 8 * (size_t)n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const int64_t done = now_ns();
    latency_ns[i] = done - (t0 + arrival_ns[i]);
    if (span_ns && i == nreq - 1) *span_ns = done - (t0 + arrival_ns[0]);
  }
  if (st) (void)hipStreamSynchronize(st);
  for (void* p : {(void*)dd, (void*)doff, (void*)df, (void*)de, (void*)ws})
    if (p) (void)hipFree(p);
  if (st) (void)hipStreamDestroy(st);
  return e == hipSuccess ? UTF8V_OK : UTF8V_EHIP;
}

}  // extern "C"
