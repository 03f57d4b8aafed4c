// C-ABI of the gfx950 validator library (declared in include/utf8v.h).
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/utf8v.h"
#include "common.hpp"

// Cross-wave slots of the batch kernel for utf8v_validate_batch_noalloc: one 64-bit word
// per wave of the persistent grid (CUs x batch waves per CU), all zero when idle.  The
// loader zero-fills the array and every finished launch leaves it zero again.  Host
// code never uses this name as an address: each device's copy is reached through the
// pointer hipGetSymbolAddress gives for it.
constexpr int kScratchWords = 16384;  // 256 CUs x 64 waves per CU
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

namespace {

using utf8v::kNone;

thread_local int g_last_status = UTF8V_OK;
thread_local int g_last_hip = 0;

std::mutex g_mu;
utf8v_config g_cfg = {4, 20, 1, 16, 1, 4};

constexpr int kBatchSlotsPerCu = 64;  // = the largest batch_waves_per_cu

struct Workspace {
  unsigned long long* dmin = nullptr;  // device: scratch words (result, flag)
  unsigned long long* state = nullptr; // device: single-buffer state words (idle = kPosNone)
  int64_t* result = nullptr;           // device: first-error offset of the last call
  int* flag = nullptr;                 // device: scratch flag (offset checks)
  int64_t* host = nullptr;             // pinned host copy of result / flag
  unsigned long long* slot = nullptr;  // device: batch cross-wave slots (self-cleaning), kBatchSlotsPerCu per CU
  std::mutex mu;
  // graph-replayed batch launches: a one-node graph whose arguments are set before each replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  int graph_waves = 0, graph_cus = 0, graph_ascii = -1;
};

std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;
std::map<int, int> g_cus;

int set_status(int s) { g_last_status = s; return s; }

int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  (void)hipGetLastError();
  return set_status(e == hipErrorOutOfMemory ? UTF8V_ENOMEM : UTF8V_EHIP);
}

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  return e == hipSuccess ? UTF8V_OK : hip_fail(e);
}

int num_cus_of(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cus.find(dev);
  if (it != g_cus.end()) return it->second;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    v = 0;
  }
  g_cus[dev] = v;
  return v;
}

void free_workspace(Workspace& w) {
  if (w.exec) (void)hipGraphExecDestroy(w.exec);
  if (w.graph) (void)hipGraphDestroy(w.graph);
  if (w.slot) (void)hipFree(w.slot);
  if (w.state) (void)hipFree(w.state);
  if (w.dmin) (void)hipFree(w.dmin);
  if (w.host) (void)hipHostFree(w.host);
}

// Workspace of (current device, stream); created on first use with dmin = none and
// empty batch slots (the initialisation is enqueued on the stream).
int workspace(hipStream_t st, Workspace** out) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  const int cus = num_cus_of(dev) > 0 ? num_cus_of(dev) : 1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dev, st);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) { *out = it->second.get(); return UTF8V_OK; }
  std::unique_ptr<Workspace> w(new Workspace);
  const int slots = cus * kBatchSlotsPerCu;
  hipError_t e = hipMalloc(&w->dmin, 64);
  if (e == hipSuccess) e = hipHostMalloc(&w->host, 64, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(&w->slot, sizeof(unsigned long long) * slots);
  if (e == hipSuccess) e = hipMalloc(&w->state, sizeof(unsigned long long) * utf8v::kStateWords);
  if (e == hipSuccess) {
    const std::vector<unsigned long long> idle(utf8v::kStateWords, utf8v::kPosNone);
    e = hipMemcpy(w->state, idle.data(), sizeof(unsigned long long) * idle.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    w->result = reinterpret_cast<int64_t*>(w->dmin) + 1;
    w->flag = reinterpret_cast<int*>(w->dmin + 2);
    const unsigned long long init[3] = {utf8v::kPosNone, 0, 0};
    e = hipMemcpy(w->dmin, init, sizeof init, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = utf8v::launch_batch_slots_init(w->slot, slots, st);
  if (e == hipSuccess) {
    utf8v::batch_launch_queries();
    utf8v::single_launch_queries();
  }
  if (e != hipSuccess) {
    free_workspace(*w);
    return hip_fail(e);
  }
  *out = w.get();
  g_ws.emplace(key, std::move(w));
  return UTF8V_OK;
}


// 0 if the GPU can dereference p, else UTF8V_ENOTDEVICE.
int check_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_status(UTF8V_ENOTDEVICE);
  }
  if (attr.type == hipMemoryTypeUnregistered) return set_status(UTF8V_ENOTDEVICE);
  return UTF8V_OK;
}

utf8v::TuneSingle tune_single() {
  std::lock_guard<std::mutex> lk(g_mu);
  utf8v::TuneSingle t;
  t.unroll = g_cfg.unroll;
  t.waves_per_cu = g_cfg.waves_per_cu;
  t.ascii = g_cfg.ascii;
  return t;
}

utf8v::TuneBatch tune_batch() {
  std::lock_guard<std::mutex> lk(g_mu);
  utf8v::TuneBatch t;
  t.waves_per_cu = g_cfg.batch_waves_per_cu;
  t.ascii = g_cfg.batch_ascii;
  t.unroll = g_cfg.batch_unroll;
  return t;
}

int enqueue_single(const uint8_t* buf, size_t len, int64_t* dev_out, hipStream_t st, Workspace** ws_out) {
  if ((buf == nullptr && len != 0) || (uint64_t)len >= utf8v::kPosNone) return set_status(UTF8V_EINVAL);
  if (len != 0) {
    int rc = check_device_ptr(buf);
    if (rc) return rc;
  }
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = num_cus_of(dev);
  hipError_t e = utf8v::launch_single(buf, (uint64_t)len, ws->state, dev_out ? dev_out : ws->result, tune_single(),
                                      cus > 0 ? cus : 1, st);
  if (e != hipSuccess) return hip_fail(e);
  if (ws_out) *ws_out = ws;
  return set_status(UTF8V_OK);
}

// Per device: the address of its copy of `scratch`, and its CU count, found once at the
// first allocation-free call on the device (with the device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};
int g_scratch_cus[kMaxDevices] = {};

int scratch_of(int dev, unsigned long long** ptr, int* cus) {
  if (dev < 0 || dev >= kMaxDevices) return set_status(UTF8V_EINVAL);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    unsigned long long* p = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
    utf8v::batch_launch_queries();
    g_scratch_cus[dev] = v > 0 ? v : 1;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *cus = g_scratch_cus[dev];
  return UTF8V_OK;
}

}  // namespace

extern "C" {

int utf8v_validate_batch_noalloc(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                                 int64_t* out_first_err, void* stream) {
  if (n < 0 || n > utf8v::kMaxBatchStrings) return set_status(UTF8V_EINVAL);
  if (n == 0) return set_status(UTF8V_OK);
  if (!data || !offsets || !out_flags || !out_first_err) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)data, (const void*)offsets, (const void*)out_flags, (const void*)out_first_err}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  unsigned long long* slots = nullptr;
  int cus = 0;
  rc = scratch_of(dev, &slots, &cus);
  if (rc) return rc;
  const utf8v::TuneBatch cfg = tune_batch();
  if ((int64_t)cus * (int64_t)cfg.waves_per_cu > kScratchWords) return set_status(UTF8V_EINVAL);
  hipError_t e = utf8v::launch_batch(utf8v::batch_args(data, offsets, n, out_flags, out_first_err, slots), cfg, cus,
                                     reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_validate_ex(const uint8_t* buf, size_t len, int64_t* first_err, void* stream) {
  if ((buf == nullptr && len != 0) || (uint64_t)len >= utf8v::kPosNone) return set_status(UTF8V_EINVAL);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  // the kernel writes the result straight into the workspace's pinned host word (no copy
  // step after it); one synchronous call per stream at a time
  std::lock_guard<std::mutex> lk(ws->mu);
  rc = enqueue_single(buf, len, ws->host, st, &ws);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  const int64_t r = *ws->host;
  if (first_err) *first_err = r;
  set_status(UTF8V_OK);
  return r < 0 ? 1 : 0;
}

bool utf8_validate(const uint8_t* buf, size_t len) {
  return utf8v_validate_ex(buf, len, nullptr, nullptr) == 1;
}

int utf8v_validate_async(const uint8_t* buf, size_t len, int64_t* dev_first_err, void* stream) {
  if (dev_first_err == nullptr) return set_status(UTF8V_EINVAL);
  int rc = check_device_ptr(dev_first_err);
  if (rc) return rc;
  return enqueue_single(buf, len, dev_first_err, reinterpret_cast<hipStream_t>(stream), nullptr);
}

int utf8v_validate_batch_async(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                               int64_t* out_first_err, void* stream) {
  if (n < 0 || n > utf8v::kMaxBatchStrings) return set_status(UTF8V_EINVAL);
  if (n == 0) return set_status(UTF8V_OK);
  if (!data || !offsets || !out_flags || !out_first_err) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)data, (const void*)offsets, (const void*)out_flags, (const void*)out_first_err}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = num_cus_of(dev);
  const utf8v::BatchArgs a = utf8v::batch_args(data, offsets, n, out_flags, out_first_err, ws->slot);
  hipError_t e = utf8v::launch_batch(a, tune_batch(), cus > 0 ? cus : 1, st);
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8_validate_batch(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                        int64_t* out_first_err) {
  int rc = utf8v_validate_batch_async(data, offsets, n, out_flags, out_first_err, nullptr);
  if (rc) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_validate_batch_graph(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* out_flags,
                               int64_t* out_first_err, void* stream) {
  if (n < 0 || n > utf8v::kMaxBatchStrings) return set_status(UTF8V_EINVAL);
  if (n == 0) return set_status(UTF8V_OK);
  if (!data || !offsets || !out_flags || !out_first_err) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)data, (const void*)offsets, (const void*)out_flags, (const void*)out_first_err}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // a replay recorded into a caller's capture would keep this call's arguments for good
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return hip_fail(e);
  if (cs != hipStreamCaptureStatusNone) return set_status(UTF8V_EINVAL);
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = num_cus_of(dev) > 0 ? num_cus_of(dev) : 1;
  const utf8v::TuneBatch cfg = tune_batch();
  std::lock_guard<std::mutex> lk(ws->mu);
  if (!ws->exec || ws->graph_waves != cfg.waves_per_cu || ws->graph_cus != cus || ws->graph_ascii != cfg.ascii) {
    if (ws->exec) {
      e = hipStreamSynchronize(st);  // no replay of the old graph may still be running
      if (e != hipSuccess) return hip_fail(e);
      (void)hipGraphExecDestroy(ws->exec);
      (void)hipGraphDestroy(ws->graph);
      ws->exec = nullptr;
      ws->graph = nullptr;
    }
    e = utf8v::make_batch_graph(cfg, cus, &ws->graph, &ws->exec, &ws->node);
    if (e != hipSuccess) return hip_fail(e);
    ws->graph_waves = cfg.waves_per_cu;
    ws->graph_cus = cus;
    ws->graph_ascii = cfg.ascii;
  }
  // the new arguments apply to this replay on; replays already enqueued keep theirs
  e = utf8v::set_batch_graph_args(ws->exec, ws->node,
                                  utf8v::batch_args(data, offsets, n, out_flags, out_first_err, ws->slot), cfg, cus);
  if (e == hipSuccess) e = hipGraphLaunch(ws->exec, st);
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

struct utf8v_stream {
  int dev = 0;
  int64_t* dstate = nullptr;  // device: {first-error offset of the chunks, history (8 bytes), end-check result}
  int64_t* host = nullptr;    // pinned copy of dstate
  int64_t total = 0;          // bytes fed so far
};

int utf8v_stream_create(utf8v_stream** out, void* stream) {
  if (!out) return set_status(UTF8V_EINVAL);
  std::unique_ptr<utf8v_stream> s(new utf8v_stream);
  int rc = current_device(&s->dev);
  if (rc) return rc;
  hipError_t e = hipMalloc(&s->dstate, 32);
  if (e == hipSuccess) e = hipHostMalloc(&s->host, 32, hipHostMallocDefault);
  if (e == hipSuccess)
    e = utf8v::launch_stream_reset(s->dstate, reinterpret_cast<unsigned long long*>(s->dstate + 1),
                                   reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    if (s->dstate) (void)hipFree(s->dstate);
    if (s->host) (void)hipHostFree(s->host);
    return hip_fail(e);
  }
  *out = s.release();
  return set_status(UTF8V_OK);
}

int utf8v_stream_update(utf8v_stream* s, const uint8_t* chunk, size_t len, void* stream) {
  if (!s || (chunk == nullptr && len != 0) || (uint64_t)len >= utf8v::kPosNone ||
      (uint64_t)s->total + (uint64_t)len >= utf8v::kPosNone)
    return set_status(UTF8V_EINVAL);
  if (len == 0) return set_status(UTF8V_OK);
  int rc = check_device_ptr(chunk);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  rc = workspace(st, &ws);
  if (rc) return rc;
  const int cus = num_cus_of(s->dev);
  hipError_t e = utf8v::launch_stream_chunk(chunk, (uint64_t)len, ws->state, s->dstate,
                                            reinterpret_cast<unsigned long long*>(s->dstate + 1), s->total,
                                            false, true, tune_single(), cus > 0 ? cus : 1, st);
  if (e != hipSuccess) return hip_fail(e);
  s->total += (int64_t)len;
  return set_status(UTF8V_OK);
}

int utf8v_stream_finish(utf8v_stream* s, int64_t* first_err, void* stream) {
  if (!s) return set_status(UTF8V_EINVAL);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  const int cus = num_cus_of(s->dev);
  // the end check at the stream's end, on the history: an empty chunk with the end check,
  // into its own slot, so the stream can be fed further after a finish
  hipError_t e = utf8v::launch_stream_chunk(nullptr, 0, ws->state, s->dstate + 2,
                                            reinterpret_cast<unsigned long long*>(s->dstate + 1), s->total, true,
                                            false, tune_single(), cus > 0 ? cus : 1, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->host, s->dstate, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  const int64_t r = s->host[0] >= 0 ? s->host[0] : s->host[2];
  if (first_err) *first_err = r;
  set_status(UTF8V_OK);
  return r < 0 ? 1 : 0;
}

int utf8v_stream_reset(utf8v_stream* s, void* stream) {
  if (!s) return set_status(UTF8V_EINVAL);
  hipError_t e = utf8v::launch_stream_reset(s->dstate, reinterpret_cast<unsigned long long*>(s->dstate + 1),
                                            reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  s->total = 0;
  return set_status(UTF8V_OK);
}

int64_t utf8v_stream_position(const utf8v_stream* s) { return s ? s->total : -1; }

int utf8v_stream_destroy(utf8v_stream* s) {
  if (!s) return set_status(UTF8V_EINVAL);
  (void)hipFree(s->dstate);
  (void)hipHostFree(s->host);
  delete s;
  return set_status(UTF8V_OK);
}

int utf8v_copy_validate(uint8_t* dst, const uint8_t* src, size_t len, int64_t* dev_first_err, void* stream) {
  if (!dev_first_err || ((src == nullptr || dst == nullptr) && len != 0)) return set_status(UTF8V_EINVAL);
  if (len != 0 && ((reinterpret_cast<uintptr_t>(dst) ^ reinterpret_cast<uintptr_t>(src)) & 15) != 0)
    return set_status(UTF8V_EINVAL);
  if (len != 0 && reinterpret_cast<uintptr_t>(dst) < reinterpret_cast<uintptr_t>(src) + len &&
      reinterpret_cast<uintptr_t>(src) < reinterpret_cast<uintptr_t>(dst) + len)
    return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)dst, (const void*)src, (const void*)dev_first_err}) {
    if (p == nullptr) continue;
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  int rc = workspace(st, &ws);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = num_cus_of(dev);
  hipError_t e = utf8v::launch_copy_validate(dst, src, (uint64_t)len, ws->state, dev_first_err, tune_single(),
                                             cus > 0 ? cus : 1, st);
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_error_class(const uint8_t* buf, size_t len, const int64_t* dev_first_err, uint8_t* dev_class,
                      void* stream) {
  if ((buf == nullptr && len != 0) || !dev_first_err || !dev_class) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)dev_first_err, (const void*)dev_class}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  if (len != 0) {
    int rc = check_device_ptr(buf);
    if (rc) return rc;
  }
  hipError_t e = utf8v::launch_error_class_one(buf, (int64_t)len, dev_first_err, dev_class,
                                               reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_error_classes(const uint8_t* data, const int64_t* offsets, int64_t n, const int64_t* first_err,
                        uint8_t* out_class, void* stream) {
  if (n < 0) return set_status(UTF8V_EINVAL);
  if (n == 0) return set_status(UTF8V_OK);
  if (!data || !offsets || !first_err || !out_class) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)data, (const void*)offsets, (const void*)first_err, (const void*)out_class}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  const int cus = num_cus_of(dev);
  hipError_t e = utf8v::launch_error_classes(data, offsets, n, first_err, out_class, cus > 0 ? cus : 1,
                                             reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_check_offsets(const int64_t* offsets, int64_t n, void* stream) {
  if (n < 0 || offsets == nullptr) return set_status(UTF8V_EINVAL);
  int rc = check_device_ptr(offsets);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Workspace* ws = nullptr;
  rc = workspace(st, &ws);
  if (rc) return rc;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cus = num_cus_of(dev);
  std::lock_guard<std::mutex> lk(ws->mu);  // the flag and its host copy are the workspace's
  hipError_t e = hipMemsetAsync(ws->flag, 0, sizeof(int), st);
  if (e == hipSuccess) e = utf8v::launch_offsets_check(offsets, n, ws->flag, cus > 0 ? cus : 1, st);
  if (e == hipSuccess) e = hipMemcpyAsync(ws->host, ws->flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e);
  set_status(UTF8V_OK);
  return *reinterpret_cast<int*>(ws->host) ? 0 : 1;
}

int utf8v_get_config(utf8v_config* cfg) {
  if (!cfg) return set_status(UTF8V_EINVAL);
  std::lock_guard<std::mutex> lk(g_mu);
  *cfg = g_cfg;
  return set_status(UTF8V_OK);
}

int utf8v_set_config(const utf8v_config* cfg) {
  if (!cfg) return set_status(UTF8V_EINVAL);
  const bool ok = (cfg->unroll == 1 || cfg->unroll == 2 || cfg->unroll == 4 || cfg->unroll == 8) &&
                  cfg->waves_per_cu >= 1 && cfg->waves_per_cu <= 4096 && (cfg->ascii == 0 || cfg->ascii == 1) &&
                  cfg->batch_waves_per_cu >= 1 && cfg->batch_waves_per_cu <= 64 &&
                  (cfg->batch_ascii == 0 || cfg->batch_ascii == 1) &&
                  (cfg->batch_unroll == 4 || cfg->batch_unroll == 8);
  if (!ok) return set_status(UTF8V_EINVAL);
  std::lock_guard<std::mutex> lk(g_mu);
  g_cfg = *cfg;
  return set_status(UTF8V_OK);
}

int utf8v_classify(const uint8_t* buf, size_t len, uint8_t* sc, uint8_t* err, void* stream) {
  if ((buf == nullptr && len != 0) || sc == nullptr || err == nullptr) return set_status(UTF8V_EINVAL);
  for (const void* p : {(const void*)sc, (const void*)err}) {
    int rc = check_device_ptr(p);
    if (rc) return rc;
  }
  if (len) {
    int rc = check_device_ptr(buf);
    if (rc) return rc;
  }
  hipError_t e = utf8v::launch_classify(buf, (uint64_t)len, sc, err, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_read_ceiling(const uint8_t* buf, size_t len, uint32_t* dev_out, void* stream) {
  if (!buf || !dev_out || (len & 15) || (reinterpret_cast<uintptr_t>(buf) & 15)) return set_status(UTF8V_EINVAL);
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  hipError_t e = utf8v::launch_read_ceiling(buf, len, dev_out, num_cus_of(dev), reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_copy(const uint8_t* src, uint8_t* dst, size_t len, void* stream) {
  if (!src || !dst || (len & 15) || ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15))
    return set_status(UTF8V_EINVAL);
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  hipError_t e = utf8v::launch_copy(src, dst, len, num_cus_of(dev), reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e);
  return set_status(UTF8V_OK);
}

int utf8v_last_status(void) { return g_last_status; }
int utf8v_last_hip_error(void) { return g_last_hip; }

const char* utf8v_strerror(int status) {
  switch (status) {
    case UTF8V_OK: return "ok";
    case UTF8V_EINVAL: return "invalid argument";
    case UTF8V_ENOTDEVICE: return "pointer not accessible by the GPU";
    case UTF8V_EHIP: return "HIP runtime error";
    case UTF8V_ENOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

int utf8v_num_cus(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return num_cus_of(dev);
}

int utf8v_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) free_workspace(*kv.second);
  g_ws.clear();
  return set_status(UTF8V_OK);
}

}  // extern "C"
