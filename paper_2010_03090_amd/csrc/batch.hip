// Batched lookup validation of many strings given by CSR offsets, for gfx950.
//
// String k is data[offsets[k] .. offsets[k+1]).  Each string is validated as
// its own stream: the bytes before its start count as zero (section 6, "the
// previous input is filled with zero") and its end gets the end check of
// section 6.3.  Results: flags[k] = 1 if valid, first_err[k] = start of the
// first ill-formed character relative to the string start, or -1.
//
// Work is split by bytes, not by strings: the byte range [offsets[0],
// offsets[n]] is cut into 4 KiB tiles (one 16-byte chunk per lane of a
// 256-thread block) and a persistent grid gives each block a contiguous run of
// tiles, so a 64 MiB string and a million 64-byte strings load-balance alike.
//
// Per tile the block writes a byte mask of string starts into LDS (from the
// offsets falling in the tile), and each lane validates its chunk with the
// bytes of other strings masked to zero:
//   - the lookup checks of section 6.1-6.2 at position i use prev1/prev2/prev3
//     only when they belong to the string of position i;
//   - at every string boundary i, the string that ends there (the one holding
//     byte i-1) gets the end check of section 6.3 on its own last bytes.
// A lane that sees any error finds the strings concerned and lowers their
// first detection position with atomicMin; a per-string pass turns it into the
// first-error offset.
#include "common.hpp"
#include "lookup.hpp"

namespace utf8v {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kU = 4;                       // 1 KiB slabs per wave tile
constexpr int kTile = kU * 1024;            // bytes per tile (one wave)
constexpr int kMaskPad = 16;                // mask bytes kept before the tile (last 4 used)
constexpr int kOffCap = 128;                // window boundaries cached in LDS for the error path

// Arguments come by value, or from a device parameter block when pa is not null
// (graph replays: the captured launches keep pa, only the block's contents change).
__device__ __forceinline__ BatchArgs args_of(const BatchArgs& a, const BatchArgs* pa) { return pa ? *pa : a; }

__global__ void batch_init(BatchArgs a0, const BatchArgs* pa) {
  const BatchArgs a = args_of(a0, pa);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += (int64_t)gridDim.x * blockDim.x)
    a.tmp[k] = kNoneRel;
}

// First k in [0, n] with offsets[k] >= target (offsets[n] >= target is guaranteed by the caller).
__device__ int64_t wave_lower_bound(const int64_t* __restrict__ offsets, int64_t n, int64_t target, int lane) {
  int64_t lo = 0, hi = n;  // answer in [lo, hi]
  while (lo < hi) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)lane * step;
    const bool below = idx < hi && offsets[idx] < target;
    const int c = __popcll(__ballot(below));
    const int64_t new_lo = c == 0 ? lo : lo + (int64_t)(c - 1) * step + 1;
    int64_t new_hi = lo + (int64_t)c * step;
    lo = new_lo;
    hi = new_hi < hi ? new_hi : hi;
  }
  return lo;
}

// String holding position pos: the last k in [k0-1, k1-1] with offsets[k] <= pos.
// Boundaries k0..k1-1 are cached in LDS (soff) when there are at most kOffCap of them.
__device__ int64_t string_of(int64_t pos, const int64_t* __restrict__ offsets, int64_t k0, int64_t k1,
                             const int64_t* soff) {
  const bool cached = k1 - k0 <= kOffCap;
  int64_t lo = k0, hi = k1;  // first k in [k0, k1] with offsets[k] > pos
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t v = cached ? soff[mid - k0] : offsets[mid];
    if (v <= pos) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

// Bytes [q, q+4) of the batch range [lo, hi) as a dword, zero outside the range.
__device__ uint32_t range_dword(const uint8_t* __restrict__ data, int64_t q, int64_t lo, int64_t hi) {
  uint32_t v = 0;
  for (int b = 0; b < 4; ++b)
    if (q + b >= lo && q + b < hi) v |= (uint32_t)data[q + b] << (8 * b);
  return v;
}

// 16-byte chunk at c (16-byte aligned address) with bytes outside [lo, hi) zeroed.  The
// aligned 16 bytes are loaded only when one of them is in the range, so they lie in
// a page that holds batch bytes.
__device__ u32x4 edge_chunk(const uint8_t* __restrict__ data, int64_t c, int64_t lo, int64_t hi) {
  if (c + 16 <= lo || c >= hi) return u32x4{0, 0, 0, 0};
  u32x4 v = *reinterpret_cast<const u32x4*>(data + c);
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
  for (int j = 0; j < 4; ++j) {
    const int64_t q = c + 4 * j;
    int64_t a = lo - q, b = hi - q;  // keep bytes [a, b) of this dword
    a = a < 0 ? 0 : (a > 4 ? 4 : a);
    b = b < 0 ? 0 : (b > 4 ? 4 : b);
    const uint64_t keep = b > a ? (((1ull << (8 * b)) - 1) & ~((1ull << (8 * a)) - 1)) : 0ull;
    w[j] &= (uint32_t)keep;
  }
  return u32x4{w[0], w[1], w[2], w[3]};
}

__device__ __forceinline__ void note_error(int64_t* tmp, int64_t k, int64_t rel) {
  atomicMin(reinterpret_cast<unsigned long long*>(tmp + k), (unsigned long long)rel);
}

// Start offset of string k, for k in [k0-1, k1-1] (LDS when cached).
__device__ __forceinline__ int64_t string_start(int64_t k, const int64_t* __restrict__ offsets, int64_t k0, int64_t k1,
                                                const int64_t* soff) {
  return (k >= k0 && k1 - k0 <= kOffCap) ? soff[k - k0] : offsets[k];
}

// End offset of string k (the next boundary), for k in [k0-1, k1-1].
__device__ __forceinline__ int64_t string_end(int64_t k, const int64_t* __restrict__ offsets, int64_t k0, int64_t k1,
                                              const int64_t* soff) {
  return (k + 1 < k1 && k1 - k0 <= kOffCap) ? soff[k + 1 - k0] : offsets[k + 1];
}

// Loads of one tile: interior tiles read whole chunks (non-temporal); tiles at the
// edges of the batch range read through edge_chunk.
__device__ __forceinline__ void batch_load(u32x4 (&x)[kU], const uint8_t* __restrict__ data, int64_t ts, int64_t lo,
                                           int64_t hi, int lane) {
  if (ts - 4 >= lo && ts + kTile <= hi) {
#pragma unroll
    for (int u = 0; u < kU; ++u)
      x[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(data + ts + u * 1024 + lane * 16));
  } else {
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = edge_chunk(data, ts + u * 1024 + lane * 16, lo, hi);
  }
}

// One wave per workgroup; each wave validates a contiguous run of 4 KiB tiles.  The
// data and the first boundary offsets of tile t+1 are requested right after tile
// t's boundary scan, before tile t is classified, so their latency overlaps it.
__global__ __launch_bounds__(64) void batch_main(BatchArgs a0, const BatchArgs* pa) {
  const BatchArgs a = args_of(a0, pa);
  __shared__ __align__(16) uint8_t smask[kTile + kMaskPad];  // string starts at positions [ts-16, te)
  __shared__ int64_t soff[kOffCap];                           // offsets[k0 ..] of the window
  const int lane = threadIdx.x;
  const int64_t* __restrict__ offsets = a.offsets;
  const uint8_t* __restrict__ data = a.data;
  // the byte range is read on the device, so one launch shape serves any batch
  const int64_t lo = offsets[0], hi = offsets[a.n];
  const int64_t c0 = lo - (int64_t)((reinterpret_cast<uintptr_t>(data) + (uintptr_t)lo) & 15);
  // tiles cover [c0, hi]: position hi holds the end check of the last string
  const int64_t tiles = (hi + 1 - c0 + kTile - 1) / kTile;
  const int64_t per = (tiles + gridDim.x - 1) / gridDim.x;
  int64_t t = (int64_t)blockIdx.x * per;
  const int64_t t_end = t + per < tiles ? t + per : tiles;
  if (t >= t_end) return;
  int64_t k0 = wave_lower_bound(offsets, a.n, c0 + t * kTile - 4, lane);
  uint32_t carry = range_dword(data, c0 + t * kTile - 4, lo, hi);  // the dword before the first tile
  const bool lane0 = lane == 0;
  int ascii_skip = 0;

  u32x4 x[kU];
  batch_load(x, data, c0 + t * kTile, lo, hi, lane);
  int64_t v = k0 + lane <= a.n ? offsets[k0 + lane] : INT64_MAX;

  for (; t < t_end; ++t) {
    const int64_t ts = c0 + t * kTile;
    const int64_t te = ts + kTile;
    // 1. string-start mask of positions [ts-4, te) in LDS
#pragma unroll
    for (int u = 0; u < kU; ++u) reinterpret_cast<u32x4*>(smask + kMaskPad)[u * 64 + lane] = u32x4{0, 0, 0, 0};
    if (lane0) *reinterpret_cast<u32x4*>(smask) = u32x4{0, 0, 0, 0};
    __syncthreads();
    int64_t cnt = 0, cnt_next = 0;
    for (;;) {
      const bool in = v < te;
      if (in) {
        smask[v - ts + kMaskPad] = 0xFF;
        if (cnt + lane < kOffCap) soff[cnt + lane] = v;
      }
      const int c = __popcll(__ballot(in));
      cnt_next += __popcll(__ballot(v < te - 4));
      cnt += c;
      if (c < 64) break;
      const int64_t idx = k0 + cnt + lane;
      v = idx <= a.n ? offsets[idx] : INT64_MAX;
    }
    const int64_t k1 = k0 + cnt;  // boundaries of this window: [k0, k1)
    // 2. request tile t+1 (its window starts at boundary k0 + cnt_next)
    u32x4 nx[kU];
    const int64_t k0n = k0 + cnt_next;
    if (t + 1 < t_end) {
      batch_load(nx, data, te, lo, hi, lane);
      v = k0n + lane <= a.n ? offsets[k0n + lane] : INT64_MAX;
    }
    __syncthreads();
    // 3. the dword before each chunk: lane l-1's last dword (lane 0: lane 63 of the previous slab)
    uint32_t prev[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t rot = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[u].w, kDppWaveRor1, 0xF, 0xF, true);
      prev[u] = lane0 ? carry : rot;
      carry = rot;
    }
    // 4. checks; a tile that is all ASCII with an ASCII halo cannot hold an error (6.4)
    bool run = true;
    if (ascii_skip == 0) {
      uint32_t o = 0;
#pragma unroll
      for (int u = 0; u < kU; ++u) o |= x[u].x | x[u].y | x[u].z | x[u].w | prev[u];
      run = !__all((o & 0x80808080u) == 0);
      if (run) ascii_skip = 3;
    } else {
      --ascii_skip;
    }
    uint32_t bad = 0;  // bit u: slab u saw a regular or end-check error
    if (run) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const u32x4 s4 = reinterpret_cast<const u32x4*>(smask + kMaskPad)[u * 64 + lane];
        const uint32_t sp = *reinterpret_cast<const uint32_t*>(smask + kMaskPad + u * 1024 + lane * 16 - 4);
        uint32_t acc = 0, tail = 0;
        MaskedCarry c = masked_halo(prev[u], sp);
        masked_next(x[u].x, prev[u], s4.x, sp, c, acc, tail);
        masked_next(x[u].y, x[u].x, s4.y, s4.x, c, acc, tail);
        masked_next(x[u].z, x[u].y, s4.z, s4.y, c, acc, tail);
        masked_next(x[u].w, x[u].z, s4.w, s4.z, c, acc, tail);
        bad |= (acc | tail) ? (1u << u) : 0u;
      }
    }
    // 5. rare: give each error to its string (only the slabs that saw one)
    if (__builtin_expect(bad != 0, 0)) {
      int64_t cur_end = -1;  // end of the string of the last regular error noted by this lane
      for (int u = 0; u < kU; ++u) {
        if (!((bad >> u) & 1)) continue;
        const u32x4 s4 = reinterpret_cast<const u32x4*>(smask + kMaskPad)[u * 64 + lane];
        const uint32_t sp = *reinterpret_cast<const uint32_t*>(smask + kMaskPad + u * 1024 + lane * 16 - 4);
        const uint32_t xs[5] = {prev[u], x[u].x, x[u].y, x[u].z, x[u].w};
        const uint32_t ss[5] = {sp, s4.x, s4.y, s4.z, s4.w};
        MaskedCarry c = masked_halo(prev[u], sp);
        for (int j = 0; j < 4; ++j) {
          uint32_t e = 0, tl = 0;
          masked_next(xs[j + 1], xs[j], ss[j + 1], ss[j], c, e, tl);
          uint32_t any = e | tl;
          while (any) {
            const int b = __builtin_ctz(any) >> 3;
            any &= ~(0xFFu << (8 * b));
            const int64_t pos = ts + u * 1024 + lane * 16 + 4 * j + b;
            if (((tl >> (8 * b)) & 0xFF) && pos - 1 >= lo && pos <= hi) {
              // end check of the string holding byte pos-1
              const int64_t k = string_of(pos - 1, offsets, k0, k1, soff);
              if (k >= 0 && k < a.n) note_error(a.tmp, k, pos - string_start(k, offsets, k0, k1, soff));
            }
            if (((e >> (8 * b)) & 0xFF) && pos >= lo && pos < hi && pos >= cur_end) {
              // first regular error of a string (later ones in it cannot be earlier)
              const int64_t k = string_of(pos, offsets, k0, k1, soff);
              if (k >= 0 && k < a.n) {
                note_error(a.tmp, k, pos - string_start(k, offsets, k0, k1, soff));
                cur_end = string_end(k, offsets, k0, k1, soff);
              }
            }
          }
        }
      }
    }
    k0 = k0n;
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = nx[u];
    __syncthreads();
  }
}

// Per string: first detection -> first-error offset; flags.
__global__ void batch_finalize(BatchArgs a0, const BatchArgs* pa) {
  const BatchArgs a = args_of(a0, pa);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = a.tmp[k];
    if (d == kNoneRel) {
      a.flags[k] = 1;
      a.first_err[k] = -1;
      continue;
    }
    const int64_t st = a.offsets[k];
    const int64_t len = a.offsets[k + 1] - st;
    auto byte_at = [&](int64_t q) -> uint32_t { return (q >= 0 && q < len) ? a.data[st + q] : 0u; };
    int64_t s = d;
    for (int64_t q = d; q >= 0 && q >= d - 3; --q) {
      if (byte_at(q - 1) < 0xC0 && byte_at(q - 2) < 0xE0 && byte_at(q - 3) < 0xF0) { s = q; break; }
    }
    a.flags[k] = 0;
    a.first_err[k] = s;
  }
}

__global__ void offsets_check(const int64_t* __restrict__ offsets, int64_t n, int* bad) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= n; k += (int64_t)gridDim.x * blockDim.x) {
    const bool ok = k == 0 ? offsets[0] >= 0 : offsets[k] >= offsets[k - 1];
    if (!ok) atomicOr(bad, 1);
  }
}

hipError_t launch_offsets_check(const int64_t* offsets, int64_t n, int* bad, int num_cus, hipStream_t st) {
  int blocks = (int)((n + 256) / 256);
  if (blocks > num_cus * 8) blocks = num_cus * 8;
  hipLaunchKernelGGL(offsets_check, dim3(blocks), dim3(256), 0, st, offsets, n, bad);
  return hipGetLastError();
}

static BatchArgs make_args(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err) {
  BatchArgs a;
  a.data = data; a.offsets = offsets; a.n = n; a.lo = a.hi = a.c0 = 0;
  a.flags = flags; a.first_err = first_err;
  a.tmp = first_err;  // per-string detections are staged in the output array
  return a;
}

// The three kernels with fixed grids (grid-stride init/finalize, persistent main), so
// the same launches serve any batch; pa (device) overrides a when not null.
static hipError_t launch_batch_kernels(const BatchArgs& a, const BatchArgs* pa, const TuneBatch& cfg, int num_cus,
                                       hipStream_t st) {
  const int waves = num_cus * (cfg.waves_per_cu > 0 ? cfg.waves_per_cu : 1);
  const int fin_blocks = num_cus * 8;
  hipLaunchKernelGGL(batch_init, dim3(fin_blocks), dim3(256), 0, st, a, pa);
  hipLaunchKernelGGL(batch_main, dim3(waves), dim3(64), 0, st, a, pa);
  hipLaunchKernelGGL(batch_finalize, dim3(fin_blocks), dim3(256), 0, st, a, pa);
  return hipGetLastError();
}

hipError_t launch_batch(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err,
                        const TuneBatch& cfg, int num_cus, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  return launch_batch_kernels(make_args(data, offsets, n, flags, first_err), nullptr, cfg, num_cus, st);
}

hipError_t capture_batch_graph(const BatchArgs* dparams, const TuneBatch& cfg, int num_cus, hipGraphExec_t* exec) {
  hipStream_t cap = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const BatchArgs dummy = make_args(nullptr, nullptr, 0, nullptr, nullptr);
    hipError_t le = launch_batch_kernels(dummy, dparams, cfg, num_cus, cap);
    e = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  return e;
}

BatchArgs batch_args(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err) {
  return make_args(data, offsets, n, flags, first_err);
}

}  // namespace utf8v
