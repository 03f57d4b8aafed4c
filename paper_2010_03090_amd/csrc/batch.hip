// Batched lookup validation of many strings given by CSR offsets, for gfx950.
//
// String k is data[offsets[k] .. offsets[k+1]).  Each string is validated as
// its own stream: the bytes before its start count as zero (as at the start of
// any input in section 6) and its end gets the end check of section 6.3.
// Results: flags[k] = 1 if valid, first_err[k] = start of the first ill-formed
// character relative to the string start, or -1.
//
// One launch does everything.  Work is split by bytes, not by strings: the
// byte range [offsets[0], offsets[n]] is cut into wave tiles (4 or 8 KiB, a launch
// setting) and a persistent grid of one-wave workgroups gives each wave a contiguous
// run of tiles, so a 64 MiB string and a million 64-byte strings load-balance alike.
// A tile goes from global memory straight into one of the wave's two LDS buffers (the
// next tile's loads fill the other one while this tile is checked), preceded there by
// the 16 bytes before it.
//
// Per tile the wave first runs the single-buffer checks of section 6 over the tile
// as plain text (in their short form where the tile holds no byte >= 0xE0), and
// applies the end check of section 6.3 to the plain bytes before every string
// boundary in it.  Where the check at a boundary b passes, the string before b ends
// with a complete character, and then the checks at b, b+1 and b+2 give the same
// verdict whether or not the bytes before b are masked to zero; at later positions
// of the string the checks only read the string's own bytes.  So a tile with
// neither a plain error nor a failed end check holds only valid strings (the
// common case, written out directly).  Otherwise each string in the tile gets its
// first detection from three sources: the plain checks in its own range (but not
// at its first three positions when the check at its start failed), the checks at
// those three positions with the bytes before its start masked to zero, and the
// end check of section 6.3 on its own last bytes.  The plain detections are
// found by checking again only the 16-byte chunks that reported one: the
// flagged dwords go, in position order, into a short list in LDS, which each
// string searches for its first detection.
//
// A string that runs across tiles carries its first detection in wave-uniform
// registers; one that runs across waves gets a partial minimum from every wave it
// touches, in a workspace slot of the wave holding its start, and the last of
// those waves to arrive (an arrival count kept in the same 64-bit word) writes its
// result and resets the slot, so the workspace is clean again when the kernel ends.
#include "common.hpp"
#include "cross_wave_plan.hpp"
#include "lookup.hpp"

namespace utf8v {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A wave tile is U 1 KiB slabs, U = 4 or 8 (a launch setting): the plain check transposes
// four slabs at a time across the byte lanes.
constexpr int kPad = 16;                     // bytes kept before the tile in its LDS buffer
template <int U>
constexpr int kTileOf = U * 1024;            // bytes per tile (one wave)
template <int U>
constexpr int kBufOf = kPad + kTileOf<U> + 16;  // LDS buffer: the tile, and room for reads just past its end
constexpr int kGroupChunks = 16;             // 16-byte chunks checked again per pass (a dword per lane)
constexpr int32_t kNonePos = INT32_MAX;      // no detection (tile-relative positions)
constexpr int kNonTemporal = 2;              // cache policy of the tile loads: streamed once

// Pointers to global memory and LDS, typed so: every access compiles to a global (not
// flat) instruction, whose completion an LDS access never has to wait for.
template <class T>
using gptr = T __attribute__((address_space(1)))*;
template <class T>
using lptr = T __attribute__((address_space(3)))*;

struct DevArgs {
  gptr<const uint8_t> data;
  gptr<const int64_t> offsets;
  int64_t n;
  gptr<unsigned long long> slot;
  gptr<uint8_t> flags;
  gptr<int64_t> first_err;
};

// The buffers are device or pinned host memory, never LDS or scratch.
__device__ __forceinline__ DevArgs args_of(const BatchArgs& a) {
  return DevArgs{(gptr<const uint8_t>)a.data, (gptr<const int64_t>)a.offsets, a.n,
                 (gptr<unsigned long long>)a.slot, (gptr<uint8_t>)a.flags, (gptr<int64_t>)a.first_err};
}

// Wave-uniform 64-bit value kept in scalar registers.
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo32 = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi32 = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi32 << 32) | lo32);
}

// A wave-uniform address held in scalar registers as it is: per-lane accesses then add a
// 32-bit lane offset to it (one address register for every base), instead of the
// compiler keeping 64-bit per-lane addresses live across the loop.
template <class T>
__device__ __forceinline__ gptr<T> sgpr_base(gptr<T> p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (gptr<T>)v;
}

// A value kept in vector registers (the same in every lane): wave-uniform values the loop
// rarely needs, so the scalar registers hold those it needs on every tile.
template <class T>
__device__ __forceinline__ T in_vgpr(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

// 32-bit value of lane `src` (wave-uniform src).
__device__ __forceinline__ int32_t lane_at(int32_t v, int src) { return __builtin_amdgcn_readlane(v, src); }

// 64-bit value of lane `src` (wave-uniform src), e.g. boundary k of a window held by the lanes.
__device__ __forceinline__ int64_t lane_at64(int64_t v, int src) {
  const uint32_t lo32 = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi32 = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)hi32 << 32) | lo32);
}

// Lane l gets lane l-1's value (lane 0 gets `first`).
__device__ __forceinline__ int32_t from_lane_below(int32_t v, int32_t first, int lane) {
  const int32_t r = __builtin_amdgcn_mov_dpp(v, kDppWaveShr1, 0xF, 0xF, false);
  return lane == 0 ? first : r;
}

// Strings [k0, k1) are valid.  Each pass stores 64 results at a wave-uniform base.
__device__ __forceinline__ void write_valid(const DevArgs& a, int k0, int k1, int lane) {
  k0 = __builtin_amdgcn_readfirstlane(k0);
  k1 = __builtin_amdgcn_readfirstlane(k1);
  for (int k = k0; k < k1; k += 64) {
    if (lane < k1 - k) {
      sgpr_base(a.flags + k)[lane] = 1;
      sgpr_base(a.first_err + k)[lane] = -1;
    }
  }
}

// Position of boundary v relative to the tile start ts, for v >= ts - 8; positions past
// the tile only have to compare as such, so they saturate at kRelFar.
constexpr int32_t kRelFar = 1 << 30;
__device__ __forceinline__ int32_t tile_rel(int64_t v, int64_t ts) {
  const int64_t d = v - ts;
  return d < (int64_t)kRelFar ? (int32_t)d : kRelFar;
}

// Workgroups are dealt to the XCDs in turn (workgroup b runs on XCD b % kXcds), and
// each XCD has its own L2.  Numbering the waves so that each XCD's waves hold
// adjacent runs of tiles keeps the lines that neighbouring waves both read (tile
// edges, window offsets, boundary search probes) in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t logical_wave(int64_t b, int64_t g) {
  return g % kXcds ? b : (b % kXcds) * (g / kXcds) + b / kXcds;
}

// 64-bit value of lane `src` (0..63, per lane) of the wave.
__device__ __forceinline__ int64_t lane_value(int64_t x, int src) {
  const int addr = src << 2;
  const uint32_t l = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)x);
  const uint32_t h = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)h << 32) | l);
}

// k0 = the first k in [0, n] with offsets[k] >= target (offsets[n] >= target is
// guaranteed by the caller) and v = offsets[k0 + lane] (INT64_MAX past n): the window
// of boundaries that the wave's first tile scans.  Each round is one dependent load per
// lane, so the rounds are kept few.  The first (first_probe, issued before the wave's
// first tile is checked, so that its latency overlaps the checks) probes 64 indices 128
// apart around the index that the byte position suggests (string lengths are roughly
// stationary in a batch), leaving about 3000 indices or more on either side; the probe
// grid is aligned to 2048 indices, so waves with nearby starts read the same cache
// lines.  When the answer is outside the probes, 64-ary rounds narrow the remaining
// range; the last round reads the remaining at most 128 indices together with the 64
// after them, so the window needs no extra round.
constexpr int64_t kGap = 128;

struct Probe {
  int64_t g;   // first probed index (wave-uniform)
  int64_t pv;  // offsets[g + 128 * lane] (INT64_MAX past n)
};

// One unconditional load per lane (indices past n read offsets[n]; wave_window takes
// them as INT64_MAX).  For n <= kGap the value is not used.
__device__ __forceinline__ Probe first_probe(gptr<const int64_t> offsets, int64_t n, int64_t off_lo, int64_t off_hi,
                                             int64_t target, int lane) {
  double f = off_hi > off_lo ? (double)(target - off_lo) / (double)(off_hi - off_lo) : 0.0;
  f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
  int64_t g = (int64_t)(f * (double)n) - 3072;
  g = g < 0 ? 0 : g / 2048 * 2048;
  g = uniform(g > n - 1 ? n - 1 : g);  // in [0, n)
  const int64_t idx = g + (int64_t)lane * kGap;
  return Probe{g, offsets[idx < n ? idx : n]};
}

__device__ int64_t wave_window(gptr<const int64_t> offsets, int64_t n, int64_t target, int lane, const Probe& pr,
                               int64_t& v) {
  int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
  if (n > kGap) {
    const int c = __popcll(__ballot(pr.g + (int64_t)lane * kGap < n && pr.pv < target));  // probes below target
    if (c > 0) lo = pr.g + (int64_t)(c - 1) * kGap + 1;
    if (c < 64 && pr.g + (int64_t)c * kGap < n) hi = pr.g + (int64_t)c * kGap;  // that probe is >= target
  }
  while (hi - lo > kGap) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + (int64_t)lane * step;
    const int c = __popcll(__ballot(idx < hi && offsets[idx] < target));
    const int64_t new_lo = c == 0 ? lo : lo + (int64_t)(c - 1) * step + 1;
    const int64_t new_hi = lo + (int64_t)c * step;
    lo = new_lo;
    hi = new_hi < hi ? new_hi : hi;
  }
  const int64_t i0 = lo + lane;
  const int64_t w0 = i0 <= n ? offsets[i0] : INT64_MAX;
  const int64_t w1 = i0 + 64 <= n ? offsets[i0 + 64] : INT64_MAX;
  const int64_t w2 = i0 + 128 <= n ? offsets[i0 + 128] : INT64_MAX;
  const int c = __popcll(__ballot(i0 < hi && w0 < target)) + __popcll(__ballot(i0 + 64 < hi && w1 < target));
  // offsets[lo + c + lane] sits in w[(lane + c) / 64] of lane (lane + c) % 64
  const int q = c >> 6, r = c & 63;
  const int64_t wa = q == 0 ? w0 : (q == 1 ? w1 : w2), wb = q == 0 ? w1 : w2;
  const int src = (lane + r) & 63;
  const int64_t va = lane_value(wa, src), vb = lane_value(wb, src);
  v = lane + r < 64 ? va : vb;
  return lo + c;
}

// The window of boundaries k .. k+63 (INT64_MAX past n).
__device__ __forceinline__ int64_t load_window(gptr<const int64_t> offsets, int k, int n32, int lane) {
  if (k + 63 <= n32) return sgpr_base(offsets + k)[lane];
  return k + lane <= n32 ? offsets[k + lane] : INT64_MAX;
}

// The 16-byte chunk at c (16-byte aligned address), loaded only when one of its bytes
// is in the batch range [lo, hi), so that it lies in a page holding batch bytes.
__device__ __forceinline__ u32x4 edge_load(gptr<const uint8_t> data, int64_t c, int64_t lo, int64_t hi) {
  u32x4 v = u32x4{0, 0, 0, 0};
  if (c + 16 > lo && c < hi) v = *reinterpret_cast<gptr<const u32x4>>(data + c);
  return v;
}

// Bytes of chunk v (at c) outside [lo, hi) set to zero.
__device__ __forceinline__ u32x4 edge_mask(u32x4 v, int64_t c, int64_t lo, int64_t hi) {
  uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
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

// A tile whose bytes all lie in the batch range: its 1 KiB slabs go from global memory
// straight into the LDS buffer (lane l's 16 bytes of slab u to byte kPad + u*1024 + 16*l),
// read once.
template <int U>
__device__ __forceinline__ void dma_tile(gptr<const uint8_t> data, int64_t ts, uint8_t* buf, int lane) {
#pragma unroll
  for (int u = 0; u < U; ++u)
    __builtin_amdgcn_global_load_lds((gptr<const void>)(sgpr_base(data + ts + u * 1024) + lane * 16),
                                     (lptr<void>)(buf + kPad + u * 1024), 16, 0, kNonTemporal);
}

// A tile at an edge of the batch range: the chunks that hold batch bytes are read, the
// bytes outside [lo, hi) set to zero, and the result stored to the LDS buffer.
template <int U>
__device__ __forceinline__ void edge_tile(gptr<const uint8_t> data, int64_t ts, int64_t lo, int64_t hi, uint8_t* buf,
                                          int lane) {
  u32x4 x[U];
#pragma unroll
  for (int u = 0; u < U; ++u) x[u] = edge_load(data, ts + u * 1024 + lane * 16, lo, hi);
#pragma unroll
  for (int u = 0; u < U; ++u)
    reinterpret_cast<u32x4*>(buf + kPad + u * 1024)[lane] = edge_mask(x[u], ts + u * 1024 + lane * 16, lo, hi);
}

// Bytes q of a 16-bit mask with q in [a, b) (a and b are clamped to [0, 16]).
__device__ __forceinline__ uint32_t bit_range(int32_t a, int32_t b) {
  const uint32_t lo = (uint32_t)(a < 0 ? 0 : (a > 16 ? 16 : a));
  const uint32_t hi = (uint32_t)(b < 0 ? 0 : (b > 16 ? 16 : b));
  return hi > lo ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
}

// One bit per byte of an error dword: bit b set iff byte b is non-zero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t e) {
  const uint32_t t = (((e & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | e) & 0x80808080u;
  return ((t >> 7) * 0x00204081u) >> 21 & 0xFu;
}

// Section 6.3 on the plain bytes before tile position r (r >= -2): they end in an
// incomplete character (last byte >= 0xC0, second-to-last >= 0xE0, third-to-last >= 0xF0).
__device__ __forceinline__ bool incomplete_before(const uint8_t* tb, int32_t r) {
  const uint32_t b1 = tb[r - 1], b2 = tb[r - 2], b3 = tb[r - 3];  // read together
  return (b1 >= 0xC0u) | (b2 >= 0xE0u) | (b3 >= 0xF0u);
}

// The same check restricted to the string [s, r): its own last bytes only.
__device__ __forceinline__ bool incomplete_within(const uint8_t* tb, int32_t r, int32_t s) {
  const uint32_t b1 = tb[r - 1], b2 = tb[r - 2], b3 = tb[r - 3];
  return (r - 1 >= s && b1 >= 0xC0u) | (r - 2 >= s && b2 >= 0xE0u) | (r - 3 >= s && b3 >= 0xF0u);
}

// Section 6.1-6.2 at the positions s, s+1, s+2 of a string starting at s, its bytes
// before s taken as zero: bit j set iff position s+j is flagged.
__device__ __forceinline__ uint32_t masked_start_flags(const uint8_t* tb, int32_t s) {
  const uint32_t x = (uint32_t)tb[s] | (uint32_t)tb[s + 1] << 8 | (uint32_t)tb[s + 2] << 16;
  return nonzero_bytes(position_errors(x, 0u)) & 7u;
}

// First detection d (relative to the string start) -> first-error offset s (section
// 6.3 applied backwards: the latest k in [d-3, d] that does not cut a character), for
// a string of length len whose byte q is byte(q).  The six bytes before d are read at once.
template <class F>
__device__ __forceinline__ int64_t resolve_first_error(F byte, int64_t len, int64_t d) {
  uint32_t w[7];  // w[i] = byte d-i (0 outside the string)
#pragma unroll
  for (int i = 1; i <= 6; ++i) {
    const int64_t q = d - i;
    w[i] = (q >= 0 && q < len) ? byte(q) : 0u;
  }
#pragma unroll
  for (int i = 0; i <= 3; ++i)  // k = d - i
    if (d - i >= 0 && w[i + 1] < 0xC0 && w[i + 2] < 0xE0 && w[i + 3] < 0xF0) return d - i;
  return d;
}

template <class F>
__device__ __forceinline__ void write_result(const DevArgs& a, int64_t k, F byte, int64_t len, int64_t d) {
  if (d == kNoneRel) {
    a.flags[k] = 1;
    a.first_err[k] = -1;
  } else {
    a.flags[k] = 0;
    a.first_err[k] = resolve_first_error(byte, len, d);
  }
}

// Bytes of a string starting at st, read from the tile's LDS buffer where they lie in
// it or in the 16 bytes before it, else from global memory.
struct StringBytes {
  gptr<const uint8_t> data;
  const uint8_t* tb;
  int64_t st, ts;
  __device__ uint32_t operator()(int64_t q) const {
    const int64_t p = st + q;
    return p >= ts - kPad ? (uint32_t)tb[p - ts] : (uint32_t)data[p];
  }
};

// Bytes of a string held in the tile's LDS buffer from tile position s on.
struct TileBytes {
  const uint8_t* tb;
  int32_t s;
  __device__ uint32_t operator()(int64_t q) const { return tb[s + (int32_t)q]; }
};

// The runs of tiles of the waves: logical wave l gets tiles [l * per, (l + 1) * per).
struct TileRuns {
  int64_t tiles;
  int per;
  int tile;  // bytes per tile
  __device__ int wave_of(int64_t p, int64_t c0) const { return (int)((p - c0) / tile) / per; }
};

// Cross-wave slot word: arrivals in bits 40..63 and, in bits 0..39, the least partial
// first detection d stored as kSlotMask - d (0 = none; a string is shorter than 2^40 - 1
// bytes), so an idle slot is all zero and the least detection is the largest stored
// value.  One 64-bit word, so arrival and minimum are published together without a
// memory fence.
constexpr int kSlotShift = 40;
constexpr uint64_t kSlotMask = (1ull << kSlotShift) - 1;

// String k runs across waves ws < we; each of them contributes once the first detection d
// it saw in its part (kNoneRel if none), and the last to arrive writes the result and
// returns the slot to zero.  A contribution that does not lower the slot's detection
// (the usual case: none) is a plain atomic add of one arrival, so the many waves inside
// one long string do not contend in compare-and-swap loops.  A wave contributes for at
// most two strings (the one open at its start and the one open at its end), after its
// last tile; the two arrivals are in flight together.  Lane 0.
// A string across more than kFanIn + 1 waves is reported in groups (cross_wave_plan.hpp).

struct CrossWave {
  int64_t k, st, en, d;
  int ws, we;       // the string's first and last wave
  int slot;         // the slot this wave arrives at: ws, or its group's first wave
  int expect;       // arrivals that slot receives
  int top_expect;   // arrivals the string's slot (ws) receives
  uint64_t mine, old;
};

// w: the arriving wave.
__device__ __forceinline__ CrossWave cross_wave_begin(int64_t k, int64_t st, int64_t en, int64_t d, int64_t c0,
                                                      const TileRuns& runs, int w) {
  CrossWave c{k, st, en, d, 0, 0, 0, 0, 0, 0, 0};
  if (k >= 0) {
    c.ws = runs.wave_of(st, c0);
    c.we = runs.wave_of(en, c0);
    c.mine = d == kNoneRel ? 0 : kSlotMask - (uint64_t)d;
    const ArrivalPlan p = arrival_plan(c.ws, c.we, w);
    c.slot = p.slot;
    c.expect = p.expect;
    c.top_expect = p.top_expect;
  }
  return c;
}

// One arrival at a slot: an atomic add, or (lowering the detection) a compare-and-swap
// loop; returns the word before it.  `mine` becomes 0 when it does not lower the slot's
// detection (then the arrival is a plain add).
__device__ __forceinline__ uint64_t slot_arrive(gptr<unsigned long long> slot, uint64_t& mine) {
  if (mine != 0) {
    uint64_t old = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((old & kSlotMask) < mine) {
      const uint64_t nw = (old & ~kSlotMask) + (1ull << kSlotShift) + mine;
      unsigned long long seen = old;
      if (__hip_atomic_compare_exchange_strong(slot, &seen, (unsigned long long)nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT))
        return old;
      old = seen;
    }
    mine = 0;  // does not lower it: a plain arrival
  }
  return __hip_atomic_fetch_add(slot, 1ull << kSlotShift, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void cross_wave_arrive(const DevArgs& a, CrossWave& c, bool lowering) {
  if (c.k < 0 || (c.mine != 0) != lowering) return;
  c.old = slot_arrive(a.slot + c.slot, c.mine);
}

__device__ __forceinline__ void cross_wave_end(const DevArgs& a, const CrossWave& c) {
  if (c.k < 0 || (int)(c.old >> kSlotShift) + 1 != c.expect) return;
  uint64_t best = (c.old & kSlotMask) > c.mine ? (c.old & kSlotMask) : c.mine;
  __hip_atomic_exchange(a.slot + c.slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (c.slot != c.ws) {  // the last of a group: the group's arrival at the string's slot
    uint64_t m = best;
    const uint64_t old = slot_arrive(a.slot + c.ws, m);
    if ((int)(old >> kSlotShift) + 1 != c.top_expect) return;
    best = (old & kSlotMask) > m ? (old & kSlotMask) : m;
    __hip_atomic_exchange(a.slot + c.ws, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const gptr<const uint8_t> s = a.data + c.st;
  write_result(a, c.k, [s](int64_t q) { return (uint32_t)s[q]; }, c.en - c.st,
               best == 0 ? kNoneRel : (int64_t)(kSlotMask - best));
}

// The 16-byte chunks of a tile that reported a plain error: chunk q (tile position
// 16q, q = 64u + lane) is bit q of the mask m[0..U-1].  Wave-uniform.
template <int U>
struct BadChunks {
  uint64_t m[U];
  // The first chunk q' >= q with q' < q_end, or -1.
  __device__ __forceinline__ int next(int q, int q_end) const {
    for (; q < q_end; q = (q & ~63) + 64) {
      const int u = q >> 6;
      uint64_t w;
      if constexpr (U == 4)
        w = (u == 0 ? m[0] : u == 1 ? m[1] : u == 2 ? m[2] : m[3]) & (~0ull << (q & 63));
      else
        w = (u < 4 ? (u == 0 ? m[0] : u == 1 ? m[1] : u == 2 ? m[2] : m[3])
                   : (u == 4 ? m[4] : u == 5 ? m[5] : u == 6 ? m[6] : m[7])) &
            (~0ull << (q & 63));
      if (w) {
        const int r = (q & ~63) + (int)__builtin_ctzll(w);
        return r < q_end ? r : -1;
      }
    }
    return -1;
  }
};

// The single-buffer checks of a tile as plain text: bit u of the result is set when this
// lane's chunk of slab u holds a flagged position.  A tile that is all ASCII with an
// ASCII halo cannot hold an error (6.4); a tile without bytes >= 0xE0 (nor in the dword
// before each chunk) takes the short form of the checks, which flags the same positions.
template <bool ASCII, int U>
__device__ __forceinline__ uint32_t plain_check(const u32x4 (&x)[U], const uint32_t (&prev)[U], AsciiBackoff& ascii,
                                                AsciiBackoff& two) {
  if (ASCII && ascii.due()) {
    uint32_t o = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) o |= x[u].x | x[u].y | x[u].z | x[u].w | prev[u];
    const bool all_ascii = __all((o & 0x80808080u) == 0);
    ascii.result(all_ascii);
    if (all_ascii) return 0u;
  }
  bool short_form = false;
  if (two.due()) {
    uint32_t o = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) o |= ge_e0(x[u].x) | ge_e0(x[u].y) | ge_e0(x[u].z) | ge_e0(x[u].w) | ge_e0(prev[u]);
    short_form = __all((o & 0x80808080u) == 0);
    two.result(short_form);
  }
  uint32_t m = 0;
  if (short_form) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t e = two_byte_errors(x[u].x, prev[u]) | two_byte_errors(x[u].y, x[u].x) |
                         two_byte_errors(x[u].z, x[u].y) | two_byte_errors(x[u].w, x[u].z);
      m |= (e & 0x80808080u) ? 1u << u : 0u;
    }
  } else {  // byte lane j of the transposed check's result of slabs g..g+3 belongs to slab g + j
    m = nonzero_bytes(chunks4_errors(0u, x[0], x[1], x[2], x[3], prev[0], prev[1], prev[2], prev[3]));
    if constexpr (U == 8)
      m |= nonzero_bytes(chunks4_errors(0u, x[4], x[5], x[6], x[7], prev[4], prev[5], prev[6], prev[7])) << 4;
  }
  return m;
}

// A lane's 16-byte chunks of the tile in LDS (one per slab) and the dword before each.
template <int U>
__device__ __forceinline__ void read_tile(const uint8_t* tb, int lane, u32x4 (&x)[U], uint32_t (&prev)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    x[u] = reinterpret_cast<const u32x4*>(tb + u * 1024)[lane];
    prev[u] = *reinterpret_cast<const uint32_t*>(tb + u * 1024 + lane * 16 - 4);
  }
}

// One wave per workgroup; each wave validates a contiguous run of tiles.  The bytes and
// the boundary window of tile t+1 are requested right after tile t's boundary scan, so
// their latency overlaps tile t's checks.  Lane l of a window holds boundary kw + l, the
// end of string kw + l - 1 and the start of string kw + l.
template <bool ASCII, int U>
__global__ __launch_bounds__(64) void batch_main(BatchArgs a0, int level) {
  static_assert(U == 4 || U == 8, "the plain check transposes four slabs at a time");
  constexpr int kU = U;
  constexpr int kTile = kTileOf<U>;
  constexpr int kBufBytes = kBufOf<U>;
  const DevArgs a = args_of(a0);
  __shared__ __align__(16) uint8_t sbuf[2][kBufBytes];  // tile buffers: the tile at kPad, the 16 bytes before it at 0
  __shared__ uint32_t sflag[64];                         // flagged dwords of the error path: position | flags << 16
  const int lane = threadIdx.x;
  const bool lane0 = lane == 0;
  const gptr<const int64_t> offsets = a.offsets;
  const gptr<const uint8_t> data = a.data;
  // the byte range is read on the device, so one launch shape serves any batch
  const int64_t n = a.n;
  const int64_t lo = uniform(offsets[0]), hi = uniform(offsets[n]);
  const int64_t c0 = lo - (int64_t)((reinterpret_cast<uintptr_t>(data) + (uintptr_t)lo) & 15);
  // tiles cover [c0, hi]: position hi holds the end check of the last string.  Tile
  // indices are 32-bit (a batch range below 8 TiB), so the loop's comparisons stay scalar.
  const int64_t tiles64 = (hi + 1 - c0 + kTile - 1) / kTile;
  const int64_t per = (tiles64 + gridDim.x - 1) / gridDim.x;
  const int64_t t64 = logical_wave(blockIdx.x, gridDim.x) * per;
  if (t64 >= tiles64) return;
  int t = (int)t64;
  const int t_end = (int)(t64 + per < tiles64 ? t64 + per : tiles64);
  // Interior tiles (all bytes inside [lo, hi)) are loaded straight into LDS; the others
  // (the first and last tiles of the range) are read chunk by chunk and masked.
  const int64_t in_first64 = (lo - c0 + kTile - 1) / kTile;
  const int64_t in_last64 = hi - kTile - c0 >= 0 ? (hi - kTile - c0) / kTile : -1;
  const int t_in_first = (int)(in_first64 < tiles64 ? in_first64 : tiles64);
  const int t_in_last = (int)in_last64;
  const int64_t wave_lo = c0 + (int64_t)t * kTile;
  // The first tile's bytes do not depend on the boundary search: they are requested first
  // (into registers), then the search's first probe, and the tile is checked while the
  // probe is in flight.
  const bool edge0 = t < t_in_first || t > t_in_last;
  u32x4 x[kU];
  uint32_t prev[kU];
  if (!edge0) {
    const gptr<const u32x4> tile = sgpr_base(reinterpret_cast<gptr<const u32x4>>(data + wave_lo));
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = __builtin_nontemporal_load(tile + u * 64 + lane);
  } else {
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = edge_load(data, wave_lo + u * 1024 + lane * 16, lo, hi);
  }
  const u32x4 before = edge_load(data, wave_lo - 16, lo, hi);  // the 16 bytes before the first tile
  asm volatile("" ::: "memory");
  Probe pr = first_probe(offsets, n, lo, hi, wave_lo - 4, lane);
  if (edge0) {
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = edge_mask(x[u], wave_lo + u * 1024 + lane * 16, lo, hi);
  }
#pragma unroll
  for (int u = 0; u < kU; ++u) reinterpret_cast<u32x4*>(sbuf[0] + kPad + u * 1024)[lane] = x[u];
  if (lane0)
    *reinterpret_cast<u32x4*>(sbuf[0]) =
        wave_lo - 16 >= lo && wave_lo <= hi ? before : edge_mask(before, wave_lo - 16, lo, hi);
#pragma unroll
  for (int u = 0; u < kU; ++u) prev[u] = *reinterpret_cast<const uint32_t*>(sbuf[0] + kPad + u * 1024 + lane * 16 - 4);
  AsciiBackoff ascii;
  // the short form for 1- and 2-byte text, first tested on the wave's fourth tile: a wave
  // of a batch of short mixed strings has few tiles and would pay for a test in half of them
  AsciiBackoff two{3, 7};
  const uint32_t m_first = plain_check<ASCII, U>(x, prev, ascii, two);
  asm volatile("" : "+v"(pr.pv) : "v"(m_first));  // the probe's value is used after the check
  // String indices are 32-bit: a batch holds fewer than 2^31 - 64 strings (the host checks).
  const int n32 = (int)n;
  int64_t v;
  int k0 = (int)uniform(wave_window(offsets, n, wave_lo - 4, lane, pr, v));
  // The string open at the tile start: index and first detection so far.  The one open at
  // the wave start began before the wave (open_first): its result goes through the
  // cross-wave slot.  Its end is the first boundary >= the wave start (64 or more empty
  // strings may lie before it).
  int open_k;
  {
    int cb = __popcll(__ballot(tile_rel(v, wave_lo) < 0)), kbase = k0;
    int64_t vb = v;
    while (cb == 64) {
      kbase += 64;
      vb = load_window(offsets, kbase, n32, lane);
      cb = __popcll(__ballot(tile_rel(vb, wave_lo) < 0));
    }
    open_k = kbase + cb - 1;
  }
  // Start of the open string, held in vector registers (the same in every lane): the
  // scalar registers are kept for what every tile needs.
  int64_t open_st_v = open_k >= 0 ? offsets[open_k] : 0;
  bool first_tile = true;
  bool edge_cur = false;  // (the first tile's bytes are in place)
  bool open_first = true;
  int64_t open_d = kNoneRel;
  // The first string of the wave that began before it is handed to the cross-wave slot
  // after the last tile: the slot's atomic returns a value, and a wait for it in the loop
  // would also wait for the next tile's loads.
  int first_k = -1;
  int64_t first_en_v = 0, first_d_v = kNoneRel, first_st_v = 0;
  int64_t final_en_v = 0;  // end of the string open after the last tile
  // strings found valid in the previous tile, written during the next one (see step 3)
  int pend_lo = 0, pend_hi = 0;
  int b = 0;  // LDS buffer of tile t
  const int64_t lo_v = in_vgpr(lo), hi_v = in_vgpr(hi);
  PriorityLevelsT<int> levels(level != 0, t, t_end - t);
  for (; t < t_end; ++t) {
    levels.step(t);
    const int64_t ts = c0 + (int64_t)t * kTile;
    const int64_t te = ts + kTile;
    uint8_t* const buf = sbuf[b];
    uint8_t* const nbuf = sbuf[b ^ 1];
    const uint8_t* const tb = buf + kPad;  // tb[p - ts] = byte p, for p >= ts - kPad
    // 1. this tile's bytes and boundary window have arrived (requested during the previous tile)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (edge_cur) edge_tile<U>(data, ts, lo_v, hi_v, buf, lane);
    // 2. boundaries of the window [ts-4, te): [k0, k1), those in [ts, te): [kb, k1).  Lane l
    // holds boundary k0 + l, as a 32-bit position relative to ts.  A tile inside one string
    // (the window's first boundary, lane 0's, lies past it) has none, and skips this and
    // the bookkeeping of steps 5-6; a tile with 64 or more is dense: its windows after the
    // first are read in the error path.
    const bool spans = uniform(v) >= te;
    int32_t rv = kRelFar;
    int cnt = 0, cnt_next = 0, cnt_before = 0;
    if (!spans) {
      rv = tile_rel(v, ts);
      cnt = __popcll(__ballot(rv < kTile));
      cnt_next = __popcll(__ballot(rv < kTile - 4));
      cnt_before = __popcll(__ballot(rv < 0));
    }
    const bool dense = cnt == 64;
    const int k1 = k0 + cnt;
    const int kb = k0 + cnt_before;
    const int64_t vwin = v;
    if (t + 1 == t_end && !dense) final_en_v = in_vgpr(lane_at64(vwin, cnt));  // first boundary >= te
    // the tile for the checks: each lane's four 16-byte chunks and the dword before each
    read_tile<U>(tb, lane, x, prev);
    // 3. requests for tile t+1 (its bytes, its window: boundaries from k0 + cnt_next on; a
    // dense tile's comes after its error path), then the previous tile's valid strings: a
    // load's wait also waits for every store issued before it, so these stores get a
    // tile's time to complete
    bool edge_next = false;
    if (t + 1 < t_end) {
      edge_next = t + 1 < t_in_first || t + 1 > t_in_last;
      if (!edge_next) dma_tile<U>(data, te, nbuf, lane);
      if (!dense && cnt_next > 0) v = load_window(offsets, k0 + cnt_next, n32, lane);
    }
    if (lane == 63) *reinterpret_cast<u32x4*>(nbuf) = x[kU - 1];  // the 16 bytes before tile t+1
    write_valid(a, pend_lo, pend_hi, lane);
    pend_lo = pend_hi = 0;
    // 4. plain checks (the wave's first tile was checked during the boundary search)
    uint32_t m;
    if (first_tile) {
      m = m_first;
      first_tile = false;
    } else {
      m = plain_check<ASCII, U>(x, prev, ascii, two);
    }
    // 5. the end check (6.3) on the plain bytes before each boundary of the window in [ts-2, te)
    // (earlier ones belong to the previous tile)
    const bool pfail = !spans && lane < cnt && rv >= -2 && incomplete_before(tb, rv);
    const bool any_plain = __any(m != 0u);
    const bool tile_bad = any_plain || (!spans && __any(pfail));
    if (!tile_bad && spans) {
      // the open string runs on past te; no string ends here
    } else if (!tile_bad && !dense) {
      // 6. every string that ends in the tile is valid, but for the first detection the
      // open string may carry; those begun in this wave form [pend_lo, pend_hi), written
      // during the next tile
      pend_lo = pend_hi = kb;
      if (open_k >= 0 && kb < k1) {  // the open string ends here
        const int64_t en = lane_at64(vwin, cnt_before);
        if (open_first) {  // it began in an earlier wave
          first_k = open_k;
          first_en_v = in_vgpr(en);
          first_d_v = in_vgpr(open_d);
          first_st_v = open_st_v;
        } else if (open_d == kNoneRel) {
          pend_lo = open_k;  // = kb - 1
        } else if (lane0) {
          const int64_t st = uniform(open_st_v);
          write_result(a, open_k, StringBytes{data, tb, st, ts}, en - st, open_d);
        }
        open_k = -1;
      }
      if (k1 - 1 > kb) pend_hi = k1 - 1;  // strings kb .. k1-2 start and end in the tile
      if (k1 - 1 >= kb && k1 <= n32) {    // the string starting here that runs past te
        open_k = k1 - 1;
        open_first = false;
        open_d = kNoneRel;
        open_st_v = in_vgpr(lane_at64(vwin, cnt - 1));
      }
    } else {
      // 7. rare: first detections string by string, window by window (a dense tile has
      // several).  Lane l's string ends at the lane's boundary e and starts at the previous
      // one s (lane 0: the open string's start, or the last boundary of the previous window).
      BadChunks<U> bad{};
      if (any_plain) {
#pragma unroll
        for (int u = 0; u < U; ++u) bad.m[u] = in_vgpr(__ballot(m & (1u << u)));
      }
      int kw = k0;          // boundary of lane 0
      int64_t vcur = vwin;  // the lane's boundary
      int32_t e = rv;       // ... tile-relative
      bool pf = pfail;      // the end check on the plain bytes before it failed
      int32_t s_first = -kRelFar;  // (window 0: lane 0's string is the open one or ended before ts)
      bool f_first = false;
      int next_total = 0;   // boundaries before kTile - 4 over the windows
      for (int w = 0;; ++w) {
        if (w > 0) {
          vcur = load_window(offsets, kw, n32, lane);
          e = tile_rel(vcur, ts);
          pf = e >= -2 && e < kTile && incomplete_before(tb, e);
        }
        const int cw = __popcll(__ballot(e < kTile));
        next_total += __popcll(__ballot(e < kTile - 4));
        const int32_t s = from_lane_below(e, s_first, lane);
        const bool fs = from_lane_below(pf ? 1 : 0, f_first ? 1 : 0, lane) != 0;
        const int kl = kw + lane;  // the lane's boundary; its string is kl - 1
        const bool active = kl >= 1 && kl <= n32 && e >= 0 && s < kTile;
        int32_t dpos = kNonePos;
        if (active) {
          if (pf && e < kTile && e > s && incomplete_within(tb, e, s)) dpos = e;
          if (fs) {  // s >= -2: positions s .. s+2 with the bytes before s masked
            const uint32_t f = masked_start_flags(tb, s) & bit_range(-s, (e < kTile ? e : kTile) - s);
            if (f) dpos = s + (int32_t)__builtin_ctz(f);
          }
        }
        // plain detections in [a0, b0): the flagged dwords of the chunks that reported one
        const int32_t a0 = (fs ? s + 3 : s) < 0 ? 0 : (fs ? s + 3 : s);
        const int32_t b0 = e < kTile ? e : kTile;
        bool need = any_plain && active && a0 < b0 && dpos >= a0;
        uint64_t needm = __ballot(need);
        if (needm) {
          // the chunks from the first searching string's start to the last one's end
          const int32_t s_lo = lane_at(s, (int)__builtin_ctzll(needm));
          int q = (s_lo < 0 ? 0 : s_lo) >> 4;
          const int q_end = (lane_at(b0, 63 - (int)__builtin_clzll(needm)) + 15) >> 4;
          for (;;) {
            int my = -1, nch = 0;
            for (; nch < kGroupChunks; ++nch) {
              const int qq = bad.next(q, q_end);
              if (qq < 0) break;
              if ((lane >> 2) == nch) my = qq * 16 + (lane & 3) * 4;
              q = qq + 1;
            }
            if (nch == 0) break;
            uint32_t fl = 0;
            if (my >= 0)
              fl = nonzero_bytes(position_errors(*reinterpret_cast<const uint32_t*>(tb + my),
                                                 *reinterpret_cast<const uint32_t*>(tb + my - 4)));
            const uint64_t fm = __ballot(fl != 0u);
            if (fm) {
              if (fl) sflag[__builtin_amdgcn_mbcnt_hi((uint32_t)(fm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)fm, 0))] =
                  (uint32_t)my | fl << 16;
              const int np = __popcll(fm);
              if (need) {  // the first listed dword with a flagged position >= a0
                int i = 0, cnt_i = np;
                while (cnt_i > 0) {
                  const int h = cnt_i >> 1;
                  const uint32_t ent = sflag[i + h];
                  const int32_t last = (int32_t)(ent & 0xFFFFu) + 31 - (int32_t)__builtin_clz(ent >> 16);
                  if (last < a0) {
                    i += h + 1;
                    cnt_i -= h + 1;
                  } else {
                    cnt_i = h;
                  }
                }
                if (i < np) {
                  const uint32_t ent = sflag[i];
                  const int32_t pos = (int32_t)(ent & 0xFFFFu);
                  const uint32_t f = (ent >> 16) & bit_range(a0 - pos, 16);
                  const int32_t p = pos + (int32_t)__builtin_ctz(f);
                  if (p < b0) {
                    dpos = p;
                    need = false;
                  }
                }
              }
            }
            // later chunks only matter to strings still searching past them
            if (!__any(need && b0 > q * 16)) break;
          }
        }
        // results.  The open string (ending at boundary open_k + 1) is done wave-uniformly:
        // its start may lie many tiles back.
        const int ol = open_k >= 0 ? open_k + 1 - kw : -1;  // its lane in this window
        const bool is_open = lane == ol;
        if (active && e < kTile && !is_open) {
          const int64_t d = dpos == kNonePos ? kNoneRel : (int64_t)(dpos - s);
          write_result(a, kl - 1, TileBytes{tb, s}, e - s, d);
        }
        if (ol >= 0 && ol < 64) {
          const int32_t od = lane_at(dpos, ol);
          const int32_t oe = lane_at(e, ol);
          const bool ends = oe < kTile;
          const int64_t st = uniform(open_st_v);
          if (od != kNonePos && ts + od - st < open_d) open_d = ts + od - st;
          if (ends) {  // it ends here
            const int64_t en = ts + oe;
            if (open_first) {
              first_k = open_k;
              first_en_v = in_vgpr(en);
              first_d_v = in_vgpr(open_d);
              first_st_v = open_st_v;
            } else if (lane0) {
              write_result(a, open_k, StringBytes{data, tb, st, ts}, en - st, open_d);
            }
            open_k = -1;
          }
        }
        // the string starting in the tile that runs past te
        const uint64_t cm = __ballot(active && e >= kTile && !is_open);
        if (cm) {
          const int l = (int)__builtin_ctzll(cm);
          const int32_t so = lane_at(s, l), od = lane_at(dpos, l);
          open_k = kw + l - 1;
          open_first = false;
          open_d = od == kNonePos ? kNoneRel : (int64_t)(od - so);
          open_st_v = in_vgpr(ts + so);
        }
        if (cw < 64) {
          if (t + 1 == t_end && dense) final_en_v = in_vgpr(lane_at64(vcur, cw));  // first boundary >= te
          break;
        }
        s_first = lane_at(e, 63);
        f_first = lane_at(pf ? 1 : 0, 63) != 0;
        kw += 64;
      }
      if (dense && t + 1 < t_end) v = load_window(offsets, k0 + next_total, n32, lane);
      k0 += next_total - cnt_next;  // (with the common advance below)
    }
    k0 += cnt_next;
    edge_cur = edge_next;
    b ^= 1;
  }
  write_valid(a, pend_lo, pend_hi, lane);
  // the strings that run across waves: the one open at the wave start that ended in it,
  // and the one still open, which runs into the next wave
  if (lane0 && (first_k >= 0 || open_k >= 0)) {
    const int64_t tiles_u = (uniform(hi_v) + 1 - c0 + kTile - 1) / kTile;
    const TileRuns runs_u{tiles_u, (int)((tiles_u + gridDim.x - 1) / gridDim.x), kTile};
    const int wl = (int)logical_wave(blockIdx.x, gridDim.x);
    CrossWave c1 =
        cross_wave_begin(first_k, uniform(first_st_v), uniform(first_en_v), uniform(first_d_v), c0, runs_u, wl);
    CrossWave c2 = cross_wave_begin(open_k, uniform(open_st_v), uniform(final_en_v), open_d, c0, runs_u, wl);
    cross_wave_arrive(a, c1, false);
    cross_wave_arrive(a, c2, false);
    cross_wave_arrive(a, c1, true);
    cross_wave_arrive(a, c2, true);
    cross_wave_end(a, c1);
    cross_wave_end(a, c2);
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

// Empty cross-wave slots: no arrivals, no partial detection (all zero).
__global__ void batch_slots_init(unsigned long long* slot, int slots) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += gridDim.x * blockDim.x) slot[i] = 0ull;
}

hipError_t launch_batch_slots_init(unsigned long long* slot, int slots, hipStream_t st) {
  hipLaunchKernelGGL(batch_slots_init, dim3((slots + 255) / 256), dim3(256), 0, st, slot, slots);
  return hipGetLastError();
}

BatchArgs batch_args(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err,
                     unsigned long long* slot) {
  BatchArgs a;
  a.data = data; a.offsets = offsets; a.n = n;
  a.slot = slot;
  a.flags = flags; a.first_err = first_err;
  return a;
}

// The kernel of a launch setting: ASCII test on or off, 4 or 8 KiB tiles.
static const void* batch_kernel(const TuneBatch& cfg) {
  if (cfg.unroll == 8)
    return cfg.ascii ? reinterpret_cast<const void*>(batch_main<true, 8>)
                     : reinterpret_cast<const void*>(batch_main<false, 8>);
  return cfg.ascii ? reinterpret_cast<const void*>(batch_main<true, 4>)
                   : reinterpret_cast<const void*>(batch_main<false, 4>);
}

// One-wave workgroups of batch_main that a CU holds at once (its registers and LDS
// decide); asked once per process and kernel, when a stream's workspace is made and
// before the graph form's capture, so never while a stream is being captured.
template <bool ASCII, int U>
static int resident_waves_per_cu_t() {
  static const int resident = [] {
    int blocks = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_main<ASCII, U>, 64, 0) == hipSuccess ? blocks
                                                                                                          : 0;
  }();
  return resident;
}

static int resident_waves_per_cu(const TuneBatch& cfg) {
  if (cfg.unroll == 8) return cfg.ascii ? resident_waves_per_cu_t<true, 8>() : resident_waves_per_cu_t<false, 8>();
  return cfg.ascii ? resident_waves_per_cu_t<true, 4>() : resident_waves_per_cu_t<false, 4>();
}

// One persistent grid of one-wave workgroups: num_cus * waves_per_cu of them, whatever
// the batch (the kernel reads the byte range from the offsets).
static int batch_grid(const TuneBatch& cfg, int num_cus) {
  return num_cus * (cfg.waves_per_cu > 0 ? cfg.waves_per_cu : 1);
}

static int batch_level(const TuneBatch& cfg) {
  return (cfg.waves_per_cu > 0 ? cfg.waves_per_cu : 1) <= resident_waves_per_cu(cfg) ? 1 : 0;
}

hipError_t launch_batch(const BatchArgs& a, const TuneBatch& cfg, int num_cus, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n > kMaxBatchStrings) return hipErrorInvalidValue;
  const dim3 grid(batch_grid(cfg, num_cus)), block(64);
  const int level = batch_level(cfg);
  if (cfg.unroll == 8) {
    if (cfg.ascii)
      hipLaunchKernelGGL((batch_main<true, 8>), grid, block, 0, st, a, level);
    else
      hipLaunchKernelGGL((batch_main<false, 8>), grid, block, 0, st, a, level);
  } else {
    if (cfg.ascii)
      hipLaunchKernelGGL((batch_main<true, 4>), grid, block, 0, st, a, level);
    else
      hipLaunchKernelGGL((batch_main<false, 4>), grid, block, 0, st, a, level);
  }
  return hipGetLastError();
}

void batch_launch_queries() {
  for (int u : {4, 8})
    for (int asc : {0, 1}) {
      TuneBatch t;
      t.unroll = u;
      t.ascii = asc;
      (void)resident_waves_per_cu(t);
    }
}

// Kernel node parameters of one batch launch; args[] must stay alive while they are used.
static hipKernelNodeParams batch_node_params(void** args, const TuneBatch& cfg, int num_cus) {
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(batch_kernel(cfg));
  p.gridDim = dim3(batch_grid(cfg, num_cus));
  p.blockDim = dim3(64);
  p.sharedMemBytes = 0;
  p.kernelParams = args;
  p.extra = nullptr;
  return p;
}

// The graph stays alive as long as its executable: the node handle that later argument
// updates name belongs to it.
hipError_t make_batch_graph(const TuneBatch& cfg, int num_cus, hipGraph_t* graph, hipGraphExec_t* exec,
                            hipGraphNode_t* node) {
  batch_launch_queries();
  BatchArgs a = batch_args(nullptr, nullptr, 0, nullptr, nullptr, nullptr);
  int level = batch_level(cfg);
  void* args[] = {&a, &level};
  const hipKernelNodeParams p = batch_node_params(args, cfg, num_cus);
  *graph = nullptr;
  *exec = nullptr;
  hipError_t e = hipGraphCreate(graph, 0);
  if (e == hipSuccess) e = hipGraphAddKernelNode(node, *graph, nullptr, 0, &p);
  if (e == hipSuccess) e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
  if (e != hipSuccess && *graph) {
    (void)hipGraphDestroy(*graph);
    *graph = nullptr;
  }
  return e;
}

hipError_t set_batch_graph_args(hipGraphExec_t exec, hipGraphNode_t node, const BatchArgs& a0, const TuneBatch& cfg,
                                int num_cus) {
  BatchArgs a = a0;
  int level = batch_level(cfg);
  void* args[] = {&a, &level};
  const hipKernelNodeParams p = batch_node_params(args, cfg, num_cus);
  return hipGraphExecKernelNodeSetParams(exec, node, &p);
}

}  // namespace utf8v
