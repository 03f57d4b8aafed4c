// Single-buffer lookup validation (section 6 of Keiser & Lemire) for gfx950.
//
// Layout.  Positions are byte offsets from the buffer start.  The interior
// [i0, i1) is the largest 16-byte-aligned part of the buffer; it is cut into
// wave tiles of U KiB.  In a tile, slab u (1 KiB) is read by one
// global_load_dwordx4 per lane (lane l reads bytes 16*l .. 16*l+15 of the slab),
// so every load instruction of a wave covers 1 KiB of consecutive bytes.  The
// up-to-15-byte head and tail outside the interior are validated by the last
// wave, with the bytes outside the buffer read as zero.
//
// The three bytes before each 16-byte chunk (the paper's previous register,
// section 6.1) come from the neighbouring lane through DPP (wave_ror:1); lane 0
// takes the last dword of the previous slab, and the first slab of a wave's
// first tile reads it from memory (zero before the buffer start, section 6).
// In a full tile a lane's four chunks are transposed across the byte lanes of
// its registers (chunks4_errors), so the byte before each byte sits in the
// previous register; in a partial tile the four dwords of each chunk form a run
// whose sign masks, nibble indices and section 6.2 inputs are shifted from one
// dword into the next (errors_next).  A full tile with no byte >= 0xE0 (nor in the
// dword before each chunk) can only hold 1- and 2-byte characters; there the checks
// reduce to a short form with the same error positions (two_byte_errors), tested
// per tile with an exponential back-off.
//
// Errors are ORed into a per-lane register (the paper's error register).  Only
// when it is non-zero does a lane recompute its chunk to find its first
// detection position.  Each wave then reports its minimum and its arrival in a
// 64-bit state word (arrivals in the high bits, least position in the low 40
// bits), so no memory fence is needed; the last wave to arrive turns the
// overall first detection position d into the first-error offset s (the start
// of the first ill-formed character),
//   s = max{ k in [max(0, d-3), d] : no character is open at k },
// writes it, and returns the state words to idle for the next call.  The last
// wave also validates the head and tail chunks outside the interior and
// applies the end check (section 6.3) before its tiles.
#include "common.hpp"
#include "lookup.hpp"

namespace utf8v {

struct SingleArgs {
  const uint8_t* buf;
  uint64_t n;                 // buffer length
  uint64_t i0, i1;            // interior [i0, i1): 16-byte aligned
  uint64_t tiles, tiles_per_wave;
  unsigned long long* state;  // top word, then kStateGroups group words kStateStride apart
  int64_t* out;               // first-error offset, -1 if valid
  // Streams (a buffer that continues earlier chunks); a plain buffer has hist = null,
  // base = 0, end_check = 1, keep_first = 0.
  unsigned long long* hist;   // the 8 bytes before position 0 (byte 7 = position -1), or null (zeros)
  int64_t base;               // stream position of byte 0 (offsets written are stream positions)
  int end_check;              // apply the section 6.3 end check at position n (else positions >= n do not exist)
  int keep_first;             // leave *out alone if it already holds an error; write no -1
  uint8_t* dst;               // copy the buffer here while validating it (the copying kernel only)
  int level;                  // the whole grid is resident at once: priority levels (common.hpp)
};

// Byte at position p of a buffer whose history (positions -8..-1) is h; zero elsewhere.
__device__ __forceinline__ uint32_t byte_at(const uint8_t* __restrict__ buf, int64_t n, uint64_t h, int64_t p) {
  if (p >= 0 && p < n) return buf[p];
  if (p < 0 && p >= -8) return (uint32_t)(h >> (8 * (8 + p))) & 0xFFu;
  return 0u;
}

__device__ __forceinline__ uint64_t history(const SingleArgs& a) { return a.hist ? *a.hist : 0ull; }

// Dword of bytes [pos-4, pos), from the history below position 0.  (buf + pos) is
// 16-byte aligned.
__device__ __forceinline__ uint32_t prev_dword(const SingleArgs& a, uint64_t pos) {
  if (pos >= 4) return *reinterpret_cast<const uint32_t*>(a.buf + pos - 4);
  const uint64_t h = history(a);
  uint32_t v = 0;
  for (int j = 0; j < 4; ++j) v |= byte_at(a.buf, (int64_t)a.n, h, (int64_t)pos - 4 + j) << (8 * j);
  return v;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Streaming 16-byte load; non-temporal, the input is read exactly once.
__device__ __forceinline__ u32x4 load16(const uint8_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
}

template <int U, bool FULL>
__device__ __forceinline__ void load_tile(u32x4 (&x)[U], const uint8_t* __restrict__ buf, uint64_t base,
                                          uint64_t i1, int lane) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t pos = base + (uint64_t)u * 1024 + (uint64_t)lane * 16;
    x[u] = (FULL || pos < i1) ? load16(buf + pos) : u32x4{0, 0, 0, 0};
  }
}

// Streaming 16-byte stores of a tile (the copying kernel): the same positions in dst.
template <int U, bool FULL>
__device__ __forceinline__ void store_tile(const u32x4 (&x)[U], uint8_t* __restrict__ dst, uint64_t base,
                                           uint64_t i1, int lane) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t pos = base + (uint64_t)u * 1024 + (uint64_t)lane * 16;
    if (FULL || pos < i1) __builtin_nontemporal_store(x[u], reinterpret_cast<u32x4*>(dst + pos));
  }
}

// Whether a wave tries the comparison form for text without bytes >= 0xF0 (see
// single_tile), and the back-off of its looks for such bytes while it does not.
struct ThreeTrials {
  bool on = false;
  AsciiBackoff probe;
};

// Validate one wave tile already in registers.  `carry` (lane 0) holds the dword
// before the tile and leaves with the tile's last dword.
template <int U, bool ASCII, bool FULL>
__device__ __forceinline__ void single_tile(const u32x4 (&x)[U], uint64_t base, uint64_t i1, int lane,
                                            uint32_t& carry, uint64_t& dmin, AsciiBackoff& ascii,
                                            AsciiBackoff& two, ThreeTrials& three) {
  // previous dword of each chunk: lane l-1's last dword (lane 0: lane 63 of the previous slab)
  uint32_t prev[U];
  const bool lane0 = lane == 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t rot = (uint32_t)__builtin_amdgcn_mov_dpp((int)x[u].w, kDppWaveRor1, 0xF, 0xF, true);
    prev[u] = lane0 ? carry : rot;
    carry = rot;  // lane 0 now holds lane 63's last dword of this slab
  }
  if (ASCII) {
    // Section 6.4: when the tile and the three bytes before it are all ASCII, no
    // check can fire in it (an ASCII byte after ASCII bytes is never an error).
    if (ascii.due()) {
      uint32_t o = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) o |= x[u].x | x[u].y | x[u].z | x[u].w | prev[u];
      const bool all_ascii = __all((o & 0x80808080u) == 0);
      ascii.result(all_ascii);
      if (all_ascii) return;
    }
  }
  uint32_t acc = 0;
  if (FULL && U % 4 == 0) {
    // a tile of 1- and 2-byte characters only (no byte >= 0xE0 in it or before its
    // chunks) takes the short form of the checks; tested with the same back-off
    bool short_form = false;
    if (two.due()) {
      uint32_t o = 0;
#pragma unroll
      for (int u = 0; u < U; ++u) o |= ge_e0(x[u].x) | ge_e0(x[u].y) | ge_e0(x[u].z) | ge_e0(x[u].w) | ge_e0(prev[u]);
      short_form = __all((o & 0x80808080u) == 0);
      two.result(short_form);
    }
    if (short_form) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        acc |= two_byte_errors(x[u].x, prev[u]) | two_byte_errors(x[u].y, x[u].x);
        acc |= two_byte_errors(x[u].z, x[u].y) | two_byte_errors(x[u].w, x[u].z);
      }
      acc &= 0x80808080u;
    } else {
      // Text of characters of at most three bytes: while the tiles before had no byte >=
      // 0xF0, a tile is first tried in the comparison form; when that flags anything (an
      // error, or a byte >= 0xF0 that the form does not cover) the tile is checked again
      // with the tables.  The table form then also looks for bytes >= 0xF0, and so it does
      // now and then (with the back-off) while trials are off; finding none turns them on.
      bool clean = false;
      if (three.on) {
        uint32_t f = 0;
#pragma unroll
        for (int u = 0; u < U; u += 4)
          f = chunks4_three(f, x[u], x[u + 1], x[u + 2], x[u + 3], prev[u], prev[u + 1], prev[u + 2], prev[u + 3]);
        clean = __all((f & 0x80808080u) == 0);
      }
      if (!clean) {
        if (three.on || three.probe.due()) {
          uint32_t f_seen = 0;
#pragma unroll
          for (int u = 0; u < U; u += 4)
            acc = chunks4_errors<true>(acc, x[u], x[u + 1], x[u + 2], x[u + 3], prev[u], prev[u + 1], prev[u + 2],
                                       prev[u + 3], &f_seen);
          three.on = __all((f_seen & 0x80808080u) == 0);
          three.probe.result(three.on);
        } else {
#pragma unroll
          for (int u = 0; u < U; u += 4)
            acc = chunks4_errors(acc, x[u], x[u + 1], x[u + 2], x[u + 3], prev[u], prev[u + 1], prev[u + 2],
                                 prev[u + 3]);
        }
      }
    }
  } else {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (FULL) {
      acc = chunk_errors(acc, x[u].x, x[u].y, x[u].z, x[u].w, prev[u]);
    } else {
      const uint32_t e = chunk_errors(0u, x[u].x, x[u].y, x[u].z, x[u].w, prev[u]);
      acc |= (base + (uint64_t)u * 1024 + (uint64_t)lane * 16 < i1) ? e : 0u;
    }
  }
  }
  if (__builtin_expect(acc != 0, 0) && dmin == kNone) {
    // first detection position of this lane (exact recomputation, rare)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t pos = base + (uint64_t)u * 1024 + (uint64_t)lane * 16;
      if (!FULL && pos >= i1) continue;
      const uint32_t w[5] = {prev[u], x[u].x, x[u].y, x[u].z, x[u].w};
      for (int j = 0; j < 4; ++j) {
        const uint32_t e = position_errors(w[j + 1], w[j]);
        if (e && dmin == kNone) dmin = pos + 4 * j + first_byte(e);
      }
      if (dmin != kNone) break;
    }
  }
}

// First detection position in the head chunk [i0-16, i0), the tail chunk
// [i1, i1+16) and at the end (section 6.3), bytes before position 0 from the
// history and after the end read as zero; kNone if none.  Without the end check
// (a stream chunk) positions >= n do not exist yet.  One thread; every byte load
// is issued before any use.
__device__ uint64_t edge_detection(const SingleArgs& a) {
  const int64_t n = (int64_t)a.n, i0 = (int64_t)a.i0, i1 = (int64_t)a.i1;
  const uint64_t hv = history(a);
  auto dword_at = [&](int64_t p) -> uint32_t {
    return byte_at(a.buf, n, hv, p) | byte_at(a.buf, n, hv, p + 1) << 8 | byte_at(a.buf, n, hv, p + 2) << 16 |
           byte_at(a.buf, n, hv, p + 3) << 24;
  };
  uint32_t h[5], t[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    h[k] = i0 > 0 ? dword_at(i0 - 20 + 4 * k) : 0u;
    t[k] = i1 < n ? dword_at(i1 - 4 + 4 * k) : 0u;
  }
  const uint32_t last = dword_at(n - 4);
  const int64_t limit = a.end_check ? INT64_MAX : n;  // detections at positions >= limit do not count
  uint64_t d = kNone;
  for (int j = 0; j < 4 && i0 > 0; ++j) {
    const uint32_t e = position_errors(h[j + 1], h[j]);
    if (e) {
      const int64_t p = i0 - 16 + 4 * j + first_byte(e);
      if (p >= 0 && p < limit) d = (uint64_t)p;
      break;
    }
  }
  for (int j = 0; j < 4 && i1 < n && d == kNone; ++j) {
    const uint32_t e = position_errors(t[j + 1], t[j]);
    if (e) {
      const int64_t p = i1 + 4 * j + first_byte(e);
      if (p < limit) d = (uint64_t)p;
      break;
    }
  }
  if (a.end_check && open_at_end(last) && (uint64_t)n < d) d = (uint64_t)n;
  return d;
}

// First detection d -> first-error offset s: the latest k in [d-3, d] at which no
// character is open (bytes before position 0 from the history; the stream starts
// at position -base).
__device__ int64_t resolve_first_error(const SingleArgs& a, int64_t d) {
  const int64_t n = (int64_t)a.n;
  const uint64_t h = history(a);
  uint32_t w[7];  // w[i] = byte d-i
#pragma unroll
  for (int i = 1; i <= 6; ++i) w[i] = d - i >= -a.base ? byte_at(a.buf, n, h, d - i) : 0u;
#pragma unroll
  for (int i = 0; i <= 3; ++i)
    if (d - i >= -a.base && w[i + 1] < 0xC0 && w[i + 2] < 0xE0 && w[i + 3] < 0xF0) return d - i;
  return d;
}

// One arrival on a state word carrying `mine` (kPosNone = no detection): the
// arrival count goes up by one and the position becomes the least of both.  An
// arrival that does not lower the position is a plain atomic add; otherwise a
// compare-and-swap loop, left as soon as the word's position is no longer higher.
// Returns the word before this arrival.
__device__ __forceinline__ uint64_t arrive(unsigned long long* w, uint64_t mine) {
  if (mine != kPosNone) {
    uint64_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while ((old & kPosNone) > mine) {
      const uint64_t nw = (old & ~kPosNone) + (1ull << kStateShift) + mine;
      const uint64_t seen = atomicCAS(w, (unsigned long long)old, (unsigned long long)nw);
      if (seen == old) return old;
      old = seen;
    }
  }
  return atomicAdd(w, 1ull << kStateShift);
}

// One wave takes a contiguous run of tiles; the loads of tile t+1 are issued
// before tile t is classified, so memory and the VALU work overlap in each wave.
// Each workgroup then reports once, by whichever of its waves finishes last (the
// others exit without waiting): on one of up to kStateGroups group words
// (workgroup index modulo the group count), and the last workgroup of a group
// reports the group on the top word, so no word sees many arrivals.
template <int U, bool ASCII, bool COPY>
__global__ __launch_bounds__(256) void single_main(SingleArgs a) {
  __shared__ unsigned long long blk_min;  // least detection of the workgroup's waves so far
  __shared__ unsigned blk_done;           // waves of the workgroup that have finished
  const int lane = threadIdx.x & 63;
  // wave index, held in a scalar register: the tile counters and priority levels below follow it
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) +
                        (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
  const uint64_t W = (uint64_t)U * 1024;
  if (threadIdx.x == 0) {
    blk_min = kPosNone;
    blk_done = 0;
  }
  __syncthreads();
  uint64_t edge = kNone;  // the last wave (usually the one with the fewest tiles) also checks the edges
  if (COPY && wave == waves - 1) {  // and copies the bytes outside the interior
    const int64_t n = (int64_t)a.n, i0 = (int64_t)a.i0, i1 = (int64_t)a.i1;
    if (lane < 16 && lane < i0 && lane < n) a.dst[lane] = a.buf[lane];
    if (lane >= 16 && lane < 32 && i1 + lane - 16 < n && i1 >= i0) a.dst[i1 + lane - 16] = a.buf[i1 + lane - 16];
  }
  if (wave == waves - 1 && lane == 0) edge = edge_detection(a);
  uint64_t t = wave * a.tiles_per_wave;
  const uint64_t t_end = t + a.tiles_per_wave < a.tiles ? t + a.tiles_per_wave : a.tiles;
  uint64_t dmin = kNone;
  if (t < t_end) {
    AsciiBackoff ascii, two;
    ThreeTrials three;
    uint32_t carry = prev_dword(a, a.i0 + t * W);
    // the buffer's last tile may be partial
    const uint64_t t_full = (t_end == a.tiles && a.i0 + a.tiles * W > a.i1) ? t_end - 1 : t_end;
    if (t < t_full) {
      // two register sets in turn: one is classified while the other's loads are in flight
      u32x4 xa[U], xb[U];
      load_tile<U, true>(xa, a.buf, a.i0 + t * W, a.i1, lane);
      PriorityLevels levels(a.level != 0, t, t_full - t);
      for (; t + 1 < t_full; t += 2) {
        levels.step(t);
        load_tile<U, true>(xb, a.buf, a.i0 + (t + 1) * W, a.i1, lane);
        if (COPY) store_tile<U, true>(xa, a.dst, a.i0 + t * W, a.i1, lane);
        single_tile<U, ASCII, true>(xa, a.i0 + t * W, a.i1, lane, carry, dmin, ascii, two, three);
        if (t + 2 < t_full) load_tile<U, true>(xa, a.buf, a.i0 + (t + 2) * W, a.i1, lane);
        if (COPY) store_tile<U, true>(xb, a.dst, a.i0 + (t + 1) * W, a.i1, lane);
        single_tile<U, ASCII, true>(xb, a.i0 + (t + 1) * W, a.i1, lane, carry, dmin, ascii, two, three);
      }
      if (t < t_full) {
        if (COPY) store_tile<U, true>(xa, a.dst, a.i0 + t * W, a.i1, lane);
        single_tile<U, ASCII, true>(xa, a.i0 + t * W, a.i1, lane, carry, dmin, ascii, two, three);
        ++t;
      }
    }
    if (t < t_end) {
      u32x4 x[U];
      load_tile<U, false>(x, a.buf, a.i0 + t * W, a.i1, lane);
      if (COPY) store_tile<U, false>(x, a.dst, a.i0 + t * W, a.i1, lane);
      single_tile<U, ASCII, false>(x, a.i0 + t * W, a.i1, lane, carry, dmin, ascii, two, three);
    }
  }
  dmin = edge < dmin ? edge : dmin;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)dmin, off);
    dmin = o < dmin ? o : dmin;
  }
  if (lane != 0) return;
  // the workgroup's last wave to finish reports for all of them (no barrier: the others exit)
  atomicMin(&blk_min, (unsigned long long)(dmin < kPosNone ? dmin : kPosNone));
  const unsigned before = __hip_atomic_fetch_add(&blk_done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (before != (blockDim.x >> 6) - 1) return;
  const uint64_t mine = __hip_atomic_load(&blk_min, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
  const uint64_t blocks = gridDim.x;
  const uint64_t groups = blocks < (uint64_t)kStateGroups ? blocks : (uint64_t)kStateGroups;
  const uint64_t g = blockIdx.x % groups;
  const uint64_t gsize = blocks / groups + (g < blocks % groups ? 1 : 0);
  unsigned long long* gw = a.state + (size_t)kStateStride * (1 + g);
  const uint64_t old = arrive(gw, mine);
  if ((old >> kStateShift) != gsize - 1) return;
  // last workgroup of its group: the group's position goes to the top word
  const uint64_t gpos = (old & kPosNone) < mine ? (old & kPosNone) : mine;
  atomicExch(gw, (unsigned long long)kPosNone);
  const uint64_t top = arrive(a.state, gpos);
  if ((top >> kStateShift) != groups - 1) return;
  // last group: every workgroup has reported
  const uint64_t pos = (top & kPosNone) < gpos ? (top & kPosNone) : gpos;
  if (!a.keep_first || *a.out < 0) {
    if (pos != kPosNone) *a.out = a.base + resolve_first_error(a, (int64_t)pos);
    else if (!a.keep_first) *a.out = -1;
  }
  if (a.hist && a.n > 0) {  // the stream's last 8 bytes, for the next chunk
    const uint64_t h = *a.hist;
    uint64_t nh = 0;
    for (int j = 0; j < 8; ++j) nh |= (uint64_t)byte_at(a.buf, (int64_t)a.n, h, (int64_t)a.n - 8 + j) << (8 * j);
    *a.hist = nh;
  }
  atomicExch(a.state, (unsigned long long)kPosNone);
}

// ---- launch -----------------------------------------------------------------------------

// Waves per CU of single_main<U, ASCII, COPY> resident at once (its registers decide).
// Asked once per process, when a stream's workspace is made (single_launch_queries),
// so never while a stream is being captured.
template <int U, bool ASCII, bool COPY>
static int resident_waves() {
  static const int waves = [] {
    int blocks = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, single_main<U, ASCII, COPY>, 256, 0) == hipSuccess
               ? 4 * blocks
               : 0;
  }();
  return waves;
}

template <int U>
static void resident_waves_all() {
  (void)resident_waves<U, true, true>();
  (void)resident_waves<U, true, false>();
  (void)resident_waves<U, false, true>();
  (void)resident_waves<U, false, false>();
}

void single_launch_queries() {
  resident_waves_all<1>();
  resident_waves_all<2>();
  resident_waves_all<4>();
  resident_waves_all<8>();
}

template <int U, bool ASCII>
static hipError_t launch_single_t(SingleArgs a, int grid, int num_cus, hipStream_t st) {
  const int64_t waves = 4 * (int64_t)grid;
  if (a.dst) {
    a.level = waves <= (int64_t)num_cus * resident_waves<U, ASCII, true>() ? 1 : 0;
    hipLaunchKernelGGL((single_main<U, ASCII, true>), dim3(grid), dim3(256), 0, st, a);
  } else {
    a.level = waves <= (int64_t)num_cus * resident_waves<U, ASCII, false>() ? 1 : 0;
    hipLaunchKernelGGL((single_main<U, ASCII, false>), dim3(grid), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_single(const uint8_t* buf, uint64_t n, unsigned long long* state, int64_t* out,
                         const TuneSingle& cfg, int num_cus, hipStream_t st) {
  return launch_stream_chunk(buf, n, state, out, nullptr, 0, true, false, cfg, num_cus, st);
}

hipError_t launch_stream_chunk(const uint8_t* buf, uint64_t n, unsigned long long* state, int64_t* out,
                               unsigned long long* hist, int64_t base, bool end_check, bool keep_first,
                               const TuneSingle& cfg, int num_cus, hipStream_t st) {
  return launch_single_any(buf, nullptr, n, state, out, hist, base, end_check, keep_first, cfg, num_cus, st);
}

hipError_t launch_copy_validate(uint8_t* dst, const uint8_t* src, uint64_t n, unsigned long long* state,
                                int64_t* out, const TuneSingle& cfg, int num_cus, hipStream_t st) {
  if (((reinterpret_cast<uintptr_t>(dst) ^ reinterpret_cast<uintptr_t>(src)) & 15) != 0) return hipErrorInvalidValue;
  return launch_single_any(src, dst, n, state, out, nullptr, 0, true, false, cfg, num_cus, st);
}

hipError_t launch_single_any(const uint8_t* buf, uint8_t* dst, uint64_t n, unsigned long long* state, int64_t* out,
                             unsigned long long* hist, int64_t base, bool end_check, bool keep_first,
                             const TuneSingle& cfg, int num_cus, hipStream_t st) {
  if (n >= kPosNone) return hipErrorInvalidValue;
  const uint64_t mis = (uint64_t)(reinterpret_cast<uintptr_t>(buf) & 15);
  const uint64_t i0 = mis ? 16 - mis : 0;
  uint64_t i1 = i0;
  if (n > i0) i1 = i0 + ((n - i0) & ~uint64_t(15));
  const int U = cfg.unroll;
  const uint64_t W = (uint64_t)U * 1024;
  SingleArgs a;
  a.buf = buf; a.n = n; a.i0 = i0; a.i1 = i1; a.state = state; a.out = out;
  a.hist = hist; a.base = base; a.end_check = end_check ? 1 : 0; a.keep_first = keep_first ? 1 : 0;
  a.dst = dst;
  a.level = 0;
  a.tiles = i1 > i0 ? (i1 - i0 + W - 1) / W : 0;
  const uint64_t max_waves = (uint64_t)num_cus * (uint64_t)cfg.waves_per_cu;
  a.tiles_per_wave = (a.tiles + max_waves - 1) / max_waves;
  if (a.tiles_per_wave < (uint64_t)cfg.min_tiles_per_wave) a.tiles_per_wave = cfg.min_tiles_per_wave;
  const uint64_t waves = a.tiles ? (a.tiles + a.tiles_per_wave - 1) / a.tiles_per_wave : 1;
  const int grid = (int)((waves + 3) / 4);  // at least one workgroup: it also does the edges and the result
  const bool asc = cfg.ascii != 0;
  switch (U) {
    case 1: return asc ? launch_single_t<1, true>(a, grid, num_cus, st) : launch_single_t<1, false>(a, grid, num_cus, st);
    case 2: return asc ? launch_single_t<2, true>(a, grid, num_cus, st) : launch_single_t<2, false>(a, grid, num_cus, st);
    case 8: return asc ? launch_single_t<8, true>(a, grid, num_cus, st) : launch_single_t<8, false>(a, grid, num_cus, st);
    default: return asc ? launch_single_t<4, true>(a, grid, num_cus, st) : launch_single_t<4, false>(a, grid, num_cus, st);
  }
}

}  // namespace utf8v
