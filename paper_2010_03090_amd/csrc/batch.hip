// Batched lookup validation of many strings given by CSR offsets, for gfx950.
//
// String k is data[offsets[k] .. offsets[k+1]).  Each string is validated as
// its own stream: the bytes before its start count as zero (as at the start of
// any input in section 6) and its end gets the end check of section 6.3.  Results: flags[k] = 1 if valid, first_err[k] = start of the
// first ill-formed character relative to the string start, or -1.
//
// One launch does everything.  Work is split by bytes, not by strings: the
// byte range [offsets[0], offsets[n]] is cut into 4 KiB tiles and a persistent
// grid of one-wave workgroups gives each wave a contiguous run of tiles, so a
// 64 MiB string and a million 64-byte strings load-balance alike.
//
// Per tile the wave first runs the single-buffer checks of section 6 over the tile as
// plain text (in their short form where the tile holds no byte >= 0xE0), and applies
// the end check of section 6.3 to the bytes before every string boundary in it.  Where a boundary's end check passes, the string before it
// ends with a complete character, and then the checks at the boundary and the two
// positions after it give the same verdict whether or not the bytes of the earlier
// string are masked to zero; so a tile with neither a plain error nor a failed end
// check holds only valid strings (the common case, written out directly).  In the 1 KiB
// slabs of a tile that do hold one, per-position error bits are needed: where no failed
// end check reaches the slab, the plain checks give them (by the same agreement); the
// other slabs are checked again per string: a string-start bitmap in LDS, the lookups
// at position i using prev1/prev2/prev3 only when they belong to the string of i, and
// each string end getting the end check on its own last bytes.  Lanes that see an
// error record, per position, a bit in one of two LDS
// bitmaps (regular error / end-check error).  Then the wave writes the result of
// every string whose end lies in the tile: its first detection is the first bit in
// its own range.  A string that runs across tiles carries its first detection in a
// wave-uniform register; one that runs across waves gets a partial minimum from every
// wave it touches, in a workspace slot of the wave holding its start, and the last of
// those waves to arrive (an arrival count kept in the same 64-bit word) writes its
// result and resets the slot, so the workspace is clean again when the kernel ends.
#include "common.hpp"
#include "lookup.hpp"

namespace utf8v {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kU = 4;                       // 1 KiB slabs per wave tile (one per byte lane of the plain check)
static_assert(kU == 4, "the plain check transposes four slabs across the byte lanes");
constexpr int kTile = kU * 1024;            // bytes per tile (one wave)
constexpr int kMaskPad = 16;                // mask bytes kept before the tile (last 4 used)
constexpr int kOffCap = 128;                // window boundaries cached in LDS for the error path

// Pointers to global memory, typed so: every access compiles to a global (not flat)
// instruction, whose completion an LDS access never has to wait for.
template <class T>
using gptr = T __attribute__((address_space(1)))*;

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


// 64-bit value of lane `src` (0..63) of the wave.
__device__ __forceinline__ int64_t lane_value(int64_t x, int src) {
  const int addr = src << 2;
  const uint32_t l = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)x);
  const uint32_t h = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)h << 32) | l);
}

// k0 = the first k in [0, n] with offsets[k] >= target (offsets[n] >= target is
// guaranteed by the caller), and v = offsets[k0 + lane] (INT64_MAX past n): the
// window of boundaries that the wave's first tile scans.  Each round is one
// dependent load per lane, so the rounds are kept few: the first probes 64 indices
// 128 apart around the index that the byte position suggests (string lengths are
// roughly stationary in a batch), leaving about 3000 indices or more on either side;
// the probe grid is aligned to 2048 indices, so waves with nearby starts read the
// same cache lines.  When the answer is outside the probes, 64-ary rounds narrow the
// remaining range; the last round reads the remaining at most 128 indices together
// with the 64 after them, so the window needs no extra round.
__device__ int64_t wave_window(gptr<const int64_t> offsets, int64_t n, int64_t off_lo, int64_t off_hi,
                               int64_t target, int lane, int64_t& v) {
  constexpr int64_t kGap = 128;
  int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
  if (n > kGap) {
    double f = off_hi > off_lo ? (double)(target - off_lo) / (double)(off_hi - off_lo) : 0.0;
    f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    int64_t g = (int64_t)(f * (double)n) - 3072;
    g = g < 0 ? 0 : g / 2048 * 2048;
    g = uniform(g > n - 1 ? n - 1 : g);  // first probe, in [0, n)
    const int64_t idx = g + (int64_t)lane * kGap;
    const int c = __popcll(__ballot(idx < n && offsets[idx] < target));  // probes below target
    if (c > 0) lo = g + (int64_t)(c - 1) * kGap + 1;
    if (c < 64 && g + (int64_t)c * kGap < n) hi = g + (int64_t)c * kGap;  // that probe is >= target
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

// Start offset of string k, for k in [k0, n] (LDS when cached).
__device__ __forceinline__ int64_t boundary(int64_t k, gptr<const int64_t> offsets, int64_t k0, int64_t k1,
                                            const int64_t* soff) {
  return (k >= k0 && k < k0 + kOffCap && k < k1) ? soff[k - k0] : offsets[k];
}

// Boundary k of a window whose cnt < 64 boundaries the lanes hold (lane l: boundary
// k0 + l): a wave-uniform k is read from its lane, a per-lane k by a lane shuffle, so
// neither waits on memory.  (A read that may come from either LDS or global memory
// makes the compiler wait for every outstanding global load, the next tile's included.)
__device__ __forceinline__ int64_t window_uniform(int64_t vwin, int64_t k, int64_t k0) {
  const int l = (int)(k - k0);
  const uint32_t lo32 = __builtin_amdgcn_readlane((int)(uint32_t)vwin, l);
  const uint32_t hi32 = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)vwin >> 32), l);
  return (int64_t)(((uint64_t)hi32 << 32) | lo32);
}

// Loads of one tile: interior tiles read whole chunks (non-temporal); tiles at the
// edges of the batch range (edge: the tile or the 4 bytes before it reach outside
// [lo, hi)) read the chunks that hold batch bytes, and batch_mask clears the bytes
// outside the range (right away, or for a wave's first tile after the boundary search,
// so the loads stay in flight during it).
__device__ __forceinline__ void batch_load(u32x4 (&x)[kU], gptr<const uint8_t> data, int64_t ts, int64_t lo,
                                           int64_t hi, int lane, bool edge) {
  if (!edge) {
    const gptr<const u32x4> tile = sgpr_base(reinterpret_cast<gptr<const u32x4>>(data + ts));
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = __builtin_nontemporal_load(tile + u * 64 + lane);
  } else {
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = edge_load(data, ts + u * 1024 + lane * 16, lo, hi);
  }
}

__device__ __forceinline__ void batch_mask(u32x4 (&x)[kU], int64_t ts, int64_t lo, int64_t hi, int lane, bool edge) {
  if (edge) {
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = edge_mask(x[u], ts + u * 1024 + lane * 16, lo, hi);
  }
}

constexpr int kMaskWords = kTile / 32;       // words of one per-position error bitmap

// Bits q in [a, b) of a 16-bit chunk mask (a and b are clamped to [0, 16]).
__device__ __forceinline__ uint32_t bit_range(int64_t a, int64_t b) {
  const uint32_t lo = (uint32_t)(a < 0 ? 0 : (a > 16 ? 16 : a));
  const uint32_t hi = (uint32_t)(b < 0 ? 0 : (b > 16 ? 16 : b));
  return hi > lo ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
}

__device__ __forceinline__ bool bit_at(const uint32_t* m, int r) { return (m[r >> 5] >> (r & 31)) & 1u; }

// Which words of a bitmap hold a set bit: bit w of (nz.lo | nz.hi << 64).  Wave-uniform.
struct WordSummary {
  uint64_t lo, hi;
};

__device__ __forceinline__ WordSummary summarize(const uint32_t* m, int lane) {
  return WordSummary{__ballot(m[lane] != 0u), __ballot(m[lane + 64] != 0u)};
}

// First word index >= w whose summary bit is set, or kMaskWords.
__device__ __forceinline__ int next_word(const WordSummary& nz, int w) {
  if (w < 64) {
    const uint64_t l = nz.lo & (~0ull << w);
    if (l) return __builtin_ctzll(l);
    w = 64;
  }
  if (w >= kMaskWords) return kMaskWords;
  const uint64_t h = nz.hi & (~0ull << (w - 64));
  return h ? 64 + __builtin_ctzll(h) : kMaskWords;
}

// First set bit of m among tile positions [a, b) (0 <= a <= b <= kTile), or -1.  Only
// words flagged in the summary are read: a word strictly inside the range that holds a
// bit ends the search, so at most the two edge words are read in vain.
__device__ int first_bit(const uint32_t* m, const WordSummary& nz, int a, int b) {
  if (a >= b) return -1;
  const int wb = (b - 1) >> 5;
  for (int w = next_word(nz, a >> 5); w <= wb; w = next_word(nz, w + 1)) {
    const int base = w * 32;
    uint32_t v = m[w];
    if (a > base) v &= ~0u << (a - base);
    if (b < base + 32) v &= (1u << (b - base)) - 1u;
    if (v) return base + __builtin_ctz(v);
  }
  return -1;
}

// One bit per byte of an error dword: bit b set iff byte b is non-zero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t e) {
  const uint32_t t = (((e & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | e) & 0x80808080u;
  return ((t >> 7) * 0x00204081u) >> 21 & 0xFu;
}

// First detection d (relative) -> first-error offset s (section 6.3 applied backwards:
// the latest k in [d-3, d] that does not cut a character), for a string of length
// len whose bytes are b[0..len) (in global memory or LDS).  The six bytes before d are
// read at once.
template <class P>
__device__ __forceinline__ int64_t resolve_first_error(P b, int64_t len, int64_t d) {
  uint32_t w[7];  // w[i] = byte d-i (0 outside the string)
#pragma unroll
  for (int i = 1; i <= 6; ++i) {
    const int64_t q = d - i;
    w[i] = (q >= 0 && q < len) ? b[q] : 0u;
  }
#pragma unroll
  for (int i = 0; i <= 3; ++i)  // k = d - i
    if (d - i >= 0 && w[i + 1] < 0xC0 && w[i + 2] < 0xE0 && w[i + 3] < 0xF0) return d - i;
  return d;
}

template <class P>
__device__ __forceinline__ void write_result(const DevArgs& a, int64_t k, P b, int64_t len, int64_t d) {
  if (d == kNoneRel) {
    a.flags[k] = 1;
    a.first_err[k] = -1;
  } else {
    a.flags[k] = 0;
    a.first_err[k] = resolve_first_error(b, len, d);
  }
}

// Wave holding position p (tiles are dealt out in runs of `per`).
__device__ __forceinline__ int64_t wave_of(int64_t p, int64_t c0, int64_t per) { return (p - c0) / kTile / per; }

// Cross-wave slot word: arrivals in bits 40..63 and, in bits 0..39, the least partial
// first detection d stored as kSlotMask - d (0 = none; a string is shorter than 2^40 - 1
// bytes), so an idle slot is all zero and the least detection is the largest stored
// value.  One 64-bit word, so arrival and minimum are published together without a
// memory fence.
constexpr int kSlotShift = 40;
constexpr uint64_t kSlotMask = (1ull << kSlotShift) - 1;

// String k runs across waves ws < we; this wave contributes the first detection d it
// saw in its part (kNoneRel if none).  The last contributor writes the result and
// returns the slot to zero.  Lane 0.  A contribution that does not lower the slot's
// detection (the usual case: none) is a plain atomic add of one arrival, so the
// many waves inside one long string do not contend in compare-and-swap loops.
__device__ void cross_wave(const DevArgs& a, int64_t k, int64_t st, int64_t en, int64_t d, int64_t c0,
                           int64_t per) {
  const int64_t ws = wave_of(st, c0, per), we = wave_of(en, c0, per);
  const gptr<unsigned long long> slot = a.slot + ws;
  const uint64_t mine = d == kNoneRel ? 0 : kSlotMask - (uint64_t)d;
  uint64_t old = 0;
  bool done = false;
  if (mine != 0) {
    old = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((old & kSlotMask) < mine) {
      const uint64_t nw = (old & ~kSlotMask) + (1ull << kSlotShift) + mine;
      unsigned long long seen = old;
      if (__hip_atomic_compare_exchange_strong(slot, &seen, (unsigned long long)nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)) {
        done = true;
        break;
      }
      old = seen;
    }
  }
  if (!done) old = __hip_atomic_fetch_add(slot, 1ull << kSlotShift, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((int64_t)(old >> kSlotShift) + 1 == we - ws + 1) {
    const uint64_t prev = old & kSlotMask;
    const uint64_t best = prev > mine ? prev : mine;
    __hip_atomic_exchange(slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    write_result(a, k, a.data + st, en - st, best == 0 ? kNoneRel : (int64_t)(kSlotMask - best));
  }
}

// The tile's bytes, and the 8 before it, into LDS (sb[kMaskPad + r] = tile byte r).
__device__ __forceinline__ void stage_tile(uint8_t* sb, const u32x4 (&x)[kU], uint32_t before2, uint32_t before1,
                                           int lane) {
#pragma unroll
  for (int u = 0; u < kU; ++u) reinterpret_cast<u32x4*>(sb + kMaskPad)[u * 64 + lane] = x[u];
  if (lane == 0) *reinterpret_cast<uint2*>(sb + kMaskPad - 8) = make_uint2(before2, before1);
  __syncthreads();
}

// The end check of section 6.3 on the (plain) bytes before the string boundary at tile
// position r >= -4: the slabs whose checks it makes unreliable when it fails (those of
// positions r, r+1, r+2), else 0.  Boundaries before -2 belong to the previous tile.
__device__ __forceinline__ uint32_t end_check_slabs(const uint8_t* tile_bytes, int r) {
  if (r < -2) return 0u;
  const uint32_t b1 = tile_bytes[r - 1], b2 = tile_bytes[r - 2], b3 = tile_bytes[r - 3];  // read together
  if ((b1 < 0xC0) & (b2 < 0xE0) & (b3 < 0xF0)) return 0u;
  return (1u << ((r < 0 ? 0 : r) >> 10)) | (1u << ((r + 2 < kTile ? r + 2 : kTile - 1) >> 10));
}

// Byte masks (0xFF per set bit) of four start bits.
__device__ __forceinline__ uint32_t bits_to_bytes(uint32_t nib) { return ((nib * 0x00204081u) & 0x01010101u) * 0xFFu; }

// One wave per workgroup; each wave validates a contiguous run of tiles.  The data
// and the first boundary offsets of tile t+1 are requested right after tile t's
// boundary scan, before tile t is classified, so their latency overlaps it.
//
// A tile is first checked as plain text (the single-buffer checks, bytes of other
// strings included), and at every string boundary b in [ts-2, te) the end check of
// section 6.3 is applied to the plain bytes before b.  Where that check passes, the
// bytes before b cannot change any check at b, b+1 or b+2 (the previous character is
// complete), so the plain checks equal the per-string ones there; elsewhere they are
// the same computation.  A tile with no plain error and no failed boundary check thus
// holds only valid strings.  In the other tiles, the 1 KiB slabs holding a plain error
// or a position b..b+2 of a failed check are checked again per string (a string-start
// bitmap in LDS, the bytes of other strings masked to zero); the remaining slabs have
// no error under either form.
// Five waves per SIMD: the kernel fits 96 VGPRs (93, no scratch); left to itself the
// compiler takes 99 and four waves, which costs the resident-grid launches their
// priority levels.
template <bool ASCII>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void batch_main(BatchArgs a0, int level) {
  const DevArgs a = args_of(a0);
  __shared__ __align__(16) uint8_t sbytes[kTile + kMaskPad];  // tile positions [-16, kTile)
  __shared__ uint32_t sbits[kMaskWords + 1];                   // string starts at positions [-32, kTile)
  __shared__ int64_t soff[kOffCap];                            // offsets[k0 ..] of the window
  __shared__ uint32_t regm[kMaskWords];                        // regular error at tile position r
  __shared__ uint32_t endm[kMaskWords];                        // end-check error at tile position r
  const int lane = threadIdx.x;
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
  const int64_t wave_lo = c0 + (int64_t)t * kTile;
  regm[lane] = regm[lane + 64] = 0u;
  endm[lane] = endm[lane + 64] = 0u;
  // Tiles whose chunks and the 4 bytes before them lie inside the batch range [lo, hi)
  // read whole chunks; the others (the first and last tiles of the range) are masked.
  const int64_t in_first64 = (lo + 4 - c0 + kTile - 1) / kTile;
  const int64_t in_last64 = hi - kTile - c0 >= 0 ? (hi - kTile - c0) / kTile : -1;
  const int t_in_first = (int)(in_first64 < tiles64 ? in_first64 : tiles64);
  const int t_in_last = (int)in_last64;
  // the first tile's bytes do not depend on the boundary search: requested before it
  u32x4 x[kU];
  const bool edge0 = t < t_in_first || t > t_in_last;
  batch_load(x, data, wave_lo, lo, hi, lane, edge0);
  const u32x4 before = edge_load(data, wave_lo - 16, lo, hi);  // the 16 bytes before the first tile
  // String indices are 32-bit: a batch holds fewer than 2^31 - 64 strings (the host checks).
  const int n32 = (int)n;
  int64_t v;
  int k0 = (int)uniform(wave_window(offsets, n, lo, hi, wave_lo - 4, lane, v));
  batch_mask(x, wave_lo, lo, hi, lane, edge0);
  const u32x4 bm = wave_lo - 16 >= lo && wave_lo <= hi ? before : edge_mask(before, wave_lo - 16, lo, hi);
  uint32_t carry = bm.w;    // the dword before the first tile
  uint32_t carry2 = bm.z;   // and the one before that
  const bool lane0 = lane == 0;
  AsciiBackoff ascii;
  // the short form for 1- and 2-byte text, first tested on the wave's fourth tile: a wave
  // of a batch of short mixed strings has few tiles and would pay for a test in half of them
  AsciiBackoff two{3, 7};
  // The string open at the tile start: index, start position and first detection so far.
  // The one open at the wave start began before the wave (open_first): its result goes
  // through the cross-wave slot.
  int open_k = -2;
  bool open_first = true;
  int64_t open_st = 0, open_d = kNoneRel;
  // strings found valid in the previous tile, written during the next one (see step 2)
  int pend_lo = 0, pend_hi = 0;

  PriorityLevelsT<int> levels(level != 0, t, t_end - t);
  for (; t < t_end; ++t) {
    levels.step(t);
    const int64_t ts = c0 + (int64_t)t * kTile;
    const int64_t te = ts + kTile;
    // 1. boundaries of the window [ts-4, te): [k0, k1), those in [ts, te): [kb, k1).  Lane l
    // holds boundary k0 + l, as a 32-bit position relative to ts.  A tile inside one string
    // (the window's first boundary lies past it) has none; a tile with 64 or more is dense:
    // its boundaries are counted window by window, the first kOffCap kept in LDS.
    const int32_t rv = tile_rel(v, ts);
    int cnt = __popcll(__ballot(rv < kTile));
    int cnt_next = __popcll(__ballot(rv < kTile - 4));
    int cnt_before = __popcll(__ballot(rv < 0));
    const bool plain = cnt == 0;
    const bool dense = cnt == 64;
    if (dense) {
      soff[lane] = v;
      for (int kk = k0 + 64;; kk += 64) {
        const int idx = kk + lane;
        const int64_t w = idx <= n32 ? offsets[idx] : INT64_MAX;
        if (kk - k0 + lane < kOffCap) soff[kk - k0 + lane] = w;
        const int32_t rw = tile_rel(w, ts);
        const int c = __popcll(__ballot(rw < kTile));
        cnt += c;
        cnt_next += __popcll(__ballot(rw < kTile - 4));
        cnt_before += __popcll(__ballot(rw < 0));
        if (c < 64) break;
      }
    }
    const int k1 = k0 + cnt;
    const int kb = k0 + cnt_before;
    // a window of at most 63 boundaries is held whole by the lanes: lane l has boundary k0 + l
    const int64_t vwin = v;
    // 2. the previous tile's valid strings are written here, before tile t+1 is requested: a
    // load's wait also waits for every store issued before it, so these stores get a tile's
    // time to complete.  Then request tile t+1 (its window starts at boundary k0 + cnt_next).
    write_valid(a, pend_lo, pend_hi, lane);
    u32x4 nx[kU];
    const int k0n = k0 + cnt_next;
    if (t + 1 < t_end) {
      const bool edge1 = t + 1 < t_in_first || t + 1 > t_in_last;
      batch_load(nx, data, te, lo, hi, lane, edge1);
      batch_mask(nx, te, lo, hi, lane, edge1);
      if (!plain) {  // (plain: the same window)
        if (k0n + 63 <= n32) v = sgpr_base(offsets + k0n)[lane];
        else v = k0n + lane <= n32 ? offsets[k0n + lane] : INT64_MAX;
      }
    }
    __syncthreads();
    if (open_k == -2) {  // first tile of the wave: the string open at its start began before it
      open_k = kb - 1;
      if (open_k >= 0) open_st = uniform(offsets[open_k]);
    }
    // 3. the dword before each chunk: lane l-1's last dword (lane 0: lane 63 of the previous slab)
    uint32_t prev[kU];
    const uint32_t before_tile = carry, before2 = carry2;  // bytes [ts-4, ts) and [ts-8, ts-4)
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t rot = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[u].w, kDppWaveRor1, 0xF, 0xF, true);
      prev[u] = lane0 ? carry : rot;
      carry = rot;
    }
    carry2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[kU - 1].z, kDppWaveRor1, 0xF, 0xF, true);
    // 4. plain checks; a tile that is all ASCII with an ASCII halo cannot hold an error (6.4)
    bool run = true;
    if (ASCII && ascii.due()) {
      uint32_t o = 0;
#pragma unroll
      for (int u = 0; u < kU; ++u) o |= x[u].x | x[u].y | x[u].z | x[u].w | prev[u];
      run = !__all((o & 0x80808080u) == 0);
      ascii.result(!run);
    }
    // bit u: this lane saw a plain error in slab u; bit 4 + u: a failed end check below reaches slab u
    uint32_t m = 0;
    if (run) {
      // a tile without bytes >= 0xE0 (nor in the dword before each chunk) takes the short
      // form of the checks: the same positions are non-zero
      bool short_form = false;
      if (two.due()) {
        uint32_t o = 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) o |= ge_e0(x[u].x) | ge_e0(x[u].y) | ge_e0(x[u].z) | ge_e0(x[u].w) | ge_e0(prev[u]);
        short_form = __all((o & 0x80808080u) == 0);
        two.result(short_form);
      }
      if (short_form) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const uint32_t e = two_byte_errors(x[u].x, prev[u]) | two_byte_errors(x[u].y, x[u].x) |
                             two_byte_errors(x[u].z, x[u].y) | two_byte_errors(x[u].w, x[u].z);
          m |= (e & 0x80808080u) ? 1u << u : 0u;
        }
      } else {  // byte lane u of the transposed check's result belongs to slab u
        m = nonzero_bytes(chunks4_errors(0u, x[0], x[1], x[2], x[3], prev[0], prev[1], prev[2], prev[3]));
      }
    }
    // 5. the tile's bytes (and the 8 before it) in LDS, for the boundary checks, the per-string
    // recheck and the resolution
    const uint8_t* tile_bytes = sbytes + kMaskPad;  // tile_bytes[p - ts] = byte p, for p >= ts - 8
    if (!plain) {
      stage_tile(sbytes, x, before2, before_tile, lane);
      // 6. the end check (6.3) on the plain bytes before every string boundary in [ts-2, te).
      // A failed check at b leaves the plain checks at b, b+1 and b+2 unreliable: their slabs
      // are rechecked.
      if (!dense) {
        if (lane < cnt) m |= end_check_slabs(tile_bytes, tile_rel(vwin, ts)) << 4;
      } else {
        for (int k = k0 + lane; k - lane < k1; k += 64)
          if (k < k1) m |= end_check_slabs(tile_bytes, (int)(boundary(k, offsets, k0, k1, soff) - ts)) << 4;
      }
    }
    const bool tile_bad = __any(m != 0u);
    uint32_t slabs = 0;   // bit u: slab u needs per-position error bits (wave-uniform)
    uint32_t mslabs = 0;  // bit u: ... from the per-string (masked) checks
    if (tile_bad) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (__any((m >> u) & 1u)) slabs |= 1u << u;
        if (__any((m >> (4 + u)) & 1u)) mslabs |= 1u << u;
      }
      slabs |= mslabs;
      if (plain) stage_tile(sbytes, x, before2, before_tile, lane);
    }
    // 7. rare: per-position error bits of the failing slabs.  Where no failed end check
    // reaches a slab, its plain checks are the per-string ones (see above); the others are
    // checked with the bytes of other strings masked to zero, from a string-start bitmap.
    WordSummary nz{0, 0};
    uint32_t bad = 0;  // bit u: this lane wrote error bits for slab u
    if (tile_bad) {
      if (mslabs) {
        sbits[lane] = 0u;
        sbits[lane + 64] = 0u;
        if (lane0) sbits[kMaskWords] = 0u;
        __syncthreads();
        if (!dense) {
          if (lane < cnt) {
            const int r = (int)(vwin - ts) + 32;  // bit index, >= 28
            atomicOr(&sbits[r >> 5], 1u << (r & 31));
          }
        } else {
          for (int k = k0 + lane; k - lane < k1; k += 64) {
            if (k < k1) {
              const int64_t r = boundary(k, offsets, k0, k1, soff) - ts + 32;  // bit index, >= 28
              atomicOr(&sbits[r >> 5], 1u << (r & 31));
            }
          }
        }
        __syncthreads();
      }
#pragma unroll 1
      for (int u = 0; u < kU; ++u) {
        if (((slabs >> u) & 1u) == 0u) continue;  // no plain error and no failed end check in it
        // the lane's 16 bytes and the dword before them
        const u32x4 xv = reinterpret_cast<const u32x4*>(tile_bytes)[u * 64 + lane];
        const uint32_t pv = *reinterpret_cast<const uint32_t*>(tile_bytes + u * 1024 + lane * 16 - 4);
        uint32_t rbits = 0, ebits = 0;
        if ((mslabs >> u) & 1u) {
          const int b = u * 1024 + lane * 16 + 32;  // bit of the lane's first position
          const uint32_t s16 = (sbits[b >> 5] >> (b & 31)) & 0xFFFFu;
          const uint32_t sp4 = (b & 31) ? (sbits[b >> 5] >> 12) & 0xFu : sbits[(b >> 5) - 1] >> 28;
          const uint32_t xs[5] = {pv, xv.x, xv.y, xv.z, xv.w};
          uint32_t ss[5];
          ss[0] = bits_to_bytes(sp4);
#pragma unroll
          for (int j = 0; j < 4; ++j) ss[j + 1] = bits_to_bytes((s16 >> (4 * j)) & 0xFu);
          MaskedCarry c = masked_halo(pv, ss[0]);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            uint32_t e = 0, tl = 0;
            masked_next(xs[j + 1], xs[j], ss[j + 1], ss[j], c, e, tl);
            rbits |= nonzero_bytes(e) << (4 * j);
            ebits |= nonzero_bytes(tl) << (4 * j);
          }
        } else {
          Carry c;
          rbits = nonzero_bytes(errors_first(0u, xv.x, pv, c));
          rbits |= nonzero_bytes(errors_next(0u, xv.y, xv.x, c)) << 4;
          rbits |= nonzero_bytes(errors_next(0u, xv.z, xv.y, c)) << 8;
          rbits |= nonzero_bytes(errors_next(0u, xv.w, xv.z, c)) << 12;
        }
        if ((rbits | ebits) != 0u) {
          const int64_t base = ts + u * 1024 + lane * 16;
          if (base - 1 < lo || base + 16 > hi) {  // chunk at an edge of the batch range
            // regular bits only at positions in [lo, hi), end-check bits in [lo + 1, hi]
            rbits &= bit_range(lo - base, hi - base);
            ebits &= bit_range(lo + 1 - base, hi + 1 - base);
          }
          reinterpret_cast<uint16_t*>(regm)[u * 64 + lane] = (uint16_t)rbits;
          reinterpret_cast<uint16_t*>(endm)[u * 64 + lane] = (uint16_t)ebits;
          bad |= 1u << u;
        }
      }
      __syncthreads();
      nz = summarize(regm, lane);
    }
    // 8. results of the strings that end in this tile (end positions in [ts, te)); those found
    // valid form the range [pend_lo, pend_hi), written during the next tile
    pend_lo = pend_hi = kb;
    if (open_k >= 0) {  // the string open at ts
      const bool ends = kb < k1;
      if (tile_bad || (ends && (open_first || open_d != kNoneRel))) {
        const int64_t en = !ends ? te
                           : !dense ? window_uniform(vwin, kb, k0)
                                    : uniform(boundary(kb, offsets, k0, k1, soff));
        if (tile_bad) {
          const int r = first_bit(regm, nz, 0, (int)(en - ts));
          if (r >= 0 && ts + r - open_st < open_d) open_d = ts + r - open_st;
          if (ends && bit_at(endm, (int)(en - ts)) && en - open_st < open_d) open_d = en - open_st;
        }
        if (ends) {
          if (open_first) {  // it began in an earlier wave
            if (lane0) cross_wave(a, open_k, open_st, en, open_d, c0, per);
          } else if (open_d == kNoneRel) {
            pend_lo = open_k;  // = kb - 1, written with the tile's valid strings
          } else if (lane0) {
            write_result(a, open_k, data + open_st, en - open_st, open_d);
          }
        }
      } else if (ends) {
        pend_lo = open_k;  // valid and begun in this wave: written with the tile's valid strings
      }
      if (ends) open_k = -1;
    }
    // strings that start and end in the tile: with no error anywhere in the tile all are valid
    if (!tile_bad) pend_hi = k1 - 1 > kb ? k1 - 1 : kb;
    for (int j0 = kb; tile_bad && j0 < k1 - 1; j0 += 64) {
      const int k = j0 + lane;
      int64_t st = 0, en = 0;
      if (!dense) {  // the shuffle reads from every lane: before the branch below
        st = lane_value(vwin, (k - k0) & 63);
        en = lane_value(vwin, (k + 1 - k0) & 63);
      }
      if (k < k1 - 1) {
        if (dense) {
          st = boundary(k, offsets, k0, k1, soff);
          en = boundary(k + 1, offsets, k0, k1, soff);
        }
        int64_t d = kNoneRel;
        if (en > st) {
          const int r = first_bit(regm, nz, (int)(st - ts), (int)(en - ts));
          if (r >= 0) d = ts + r - st;
          if (bit_at(endm, (int)(en - ts)) && en - st < d) d = en - st;
        }
        write_result(a, k, tile_bytes + (st - ts), en - st, d);
      }
    }
    if (k1 - 1 >= kb && k1 <= n32) {  // the string starting here that runs past te
      open_k = k1 - 1;
      open_first = false;
      open_st = !dense ? window_uniform(vwin, open_k, k0) : uniform(boundary(open_k, offsets, k0, k1, soff));
      open_d = kNoneRel;
      if (tile_bad) {
        const int r = first_bit(regm, nz, (int)(open_st - ts), kTile);
        if (r >= 0) open_d = ts + r - open_st;
      }
    }
    // 9. clear the error bits this lane set, once every lane has read them
    if (tile_bad) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if ((bad >> u) & 1) {
          reinterpret_cast<uint16_t*>(regm)[u * 64 + lane] = 0;
          reinterpret_cast<uint16_t*>(endm)[u * 64 + lane] = 0;
        }
      }
    }
    k0 = k0n;
#pragma unroll
    for (int u = 0; u < kU; ++u) x[u] = nx[u];
    __syncthreads();
  }
  write_valid(a, pend_lo, pend_hi, lane);
  // the string still open runs into the next wave
  if (open_k >= 0 && lane0) cross_wave(a, open_k, open_st, offsets[open_k + 1], open_d, c0, per);
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

// One-wave workgroups of batch_main that a CU holds at once (its registers decide);
// asked once per process, when a stream's workspace is made and before the graph
// form's capture, so never while a stream is being captured.
template <bool ASCII>
static int resident_waves_per_cu_t() {
  static const int resident = [] {
    int blocks = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batch_main<ASCII>, 64, 0) == hipSuccess ? blocks
                                                                                                       : 0;
  }();
  return resident;
}

static int resident_waves_per_cu(bool ascii) {
  return ascii ? resident_waves_per_cu_t<true>() : resident_waves_per_cu_t<false>();
}

// One persistent grid of one-wave workgroups: num_cus * waves_per_cu of them, whatever
// the batch (the kernel reads the byte range from the offsets).
static int batch_grid(const TuneBatch& cfg, int num_cus) {
  return num_cus * (cfg.waves_per_cu > 0 ? cfg.waves_per_cu : 1);
}

static int batch_level(const TuneBatch& cfg) {
  return (cfg.waves_per_cu > 0 ? cfg.waves_per_cu : 1) <= resident_waves_per_cu(cfg.ascii != 0) ? 1 : 0;
}

hipError_t launch_batch(const BatchArgs& a, const TuneBatch& cfg, int num_cus, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  if (a.n > kMaxBatchStrings) return hipErrorInvalidValue;
  if (cfg.ascii)
    hipLaunchKernelGGL(batch_main<true>, dim3(batch_grid(cfg, num_cus)), dim3(64), 0, st, a, batch_level(cfg));
  else
    hipLaunchKernelGGL(batch_main<false>, dim3(batch_grid(cfg, num_cus)), dim3(64), 0, st, a, batch_level(cfg));
  return hipGetLastError();
}

void batch_launch_queries() {
  (void)resident_waves_per_cu(true);
  (void)resident_waves_per_cu(false);
}

// Kernel node parameters of one batch launch; args[] must stay alive while they are used.
static hipKernelNodeParams batch_node_params(void** args, const TuneBatch& cfg, int num_cus) {
  hipKernelNodeParams p{};
  p.func = cfg.ascii ? reinterpret_cast<void*>(batch_main<true>) : reinterpret_cast<void*>(batch_main<false>);
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
