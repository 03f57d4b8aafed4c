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

constexpr int kTile = 4096;                 // bytes per tile (256 lanes x 16 bytes)
constexpr int kMaskPad = 16;                // mask bytes kept before the tile (last 4 used)
constexpr int kOffCap = 1024;               // tile boundaries cached in LDS for the error path

__global__ void batch_init(int64_t* tmp, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    tmp[k] = kNoneRel;
}

// First k in [0, n] with offsets[k] >= target (offsets[n] >= target is guaranteed by the caller).
__device__ int64_t block_lower_bound(const int64_t* __restrict__ offsets, int64_t n, int64_t target, int tid) {
  int64_t lo = 0, hi = n;  // answer in [lo, hi]
  while (lo < hi) {
    const int64_t span = hi - lo;
    const int64_t step = (span + 255) / 256;
    const int64_t idx = lo + (int64_t)tid * step;
    const bool below = idx < hi && offsets[idx] < target;
    const int c = __syncthreads_count(below);
    const int64_t new_lo = c == 0 ? lo : lo + (int64_t)(c - 1) * step + 1;
    int64_t new_hi = lo + (int64_t)c * step;
    if (new_hi > hi) new_hi = hi;
    lo = new_lo;
    hi = new_hi;
  }
  return lo;
}

// String holding position pos: the last k with offsets[k] <= pos (offsets[k0-1] < window start).
__device__ int64_t string_of(int64_t pos, const int64_t* __restrict__ offsets, int64_t k0, int64_t k1,
                             const int64_t* lds_off) {
  int64_t lo = k0, hi = k1;  // first k in [k0, k1] with offsets[k] > pos
  const bool cached = k1 - k0 <= kOffCap;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t v = cached ? lds_off[mid - k0] : offsets[mid];
    if (v <= pos) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

// Lookup checks with per-string masking.  x: the chunk dword, p: the dword before it,
// s / sp: string-start masks (0xFF where a string starts) of the same two dwords.
// Returns the errors of the strings holding each position; *tail gets the end
// check of the strings ending at each position.
__device__ __forceinline__ uint32_t masked_errors(uint32_t x, uint32_t p, uint32_t s, uint32_t sp, uint32_t* tail) {
  const uint32_t s1 = align(s, sp, 3);                     // position i-1 starts a string
  const uint32_t s2 = align(s, sp, 2);                     // position i-2 starts a string
  const uint32_t prev1 = align(x, p, 3);
  const uint32_t prev2 = align(x, p, 2);
  const uint32_t prev3 = align(x, p, 1);
  const uint32_t r2 = s | s1;                              // byte i-2 is in another string
  const uint32_t r3 = r2 | s2;                             // byte i-3 is in another string
  const uint32_t p1m = prev1 & ~s;
  // classification with prev1 of the same string (zero at a string start)
  const uint32_t sh2 = (x >> 4) & 0x07070707u;
  const uint32_t sh1 = (p1m >> 4) & 0x07070707u;
  const uint32_t sl1 = p1m & 0x07070707u;
  const uint32_t neg2 = perm(x, prev1, kSignSel);
  const uint32_t neg1 = perm(p1m, p1m << 8, kSignSel);
  const uint32_t half = ((p1m >> 1) & 0x04040404u) | 0x03020100u;
  const uint32_t b1h = select_bits(neg1, perm(kB1H_HI_HI, kB1H_HI_LO, sh1), kB1H_LOW_HALF);
  const uint32_t b1l = perm(perm(kB1L_HI_HI, kB1L_HI_LO, sl1), perm(kB1L_LO_HI, kB1L_LO_LO, sl1), half);
  const uint32_t b2h = select_bits(neg2, perm(kB2H_HI_HI, kB2H_HI_LO, sh2), kB2H_LOW_HALF);
  const uint32_t sc = and3(b1h, b1l, b2h);
  const uint32_t ge_e0 = ge_mask7(prev2, 0x20202020u);     // bit 7: byte i-2 >= 0xE0
  const uint32_t ge_f0 = ge_mask7(prev3, 0x10101010u);     // bit 7: byte i-3 >= 0xF0
  const uint32_t ge_c0 = ge_mask7(prev1, 0x40404040u);     // bit 7: byte i-1 >= 0xC0
  // section 6.2 within the string of position i
  const uint32_t m23 = ((ge_e0 & ~r2) | (ge_f0 & ~r3)) & 0x80808080u;
  // section 6.3 for the string ending at i (its bytes i-1, and i-2 / i-3 when they are its own)
  *tail = (ge_c0 | (ge_e0 & ~s1) | (ge_f0 & ~(s1 | s2))) & s & 0x80808080u;
  return sc ^ m23;
}

__global__ __launch_bounds__(256) void batch_main(BatchArgs a) {
  __shared__ __align__(16) uint8_t smask[kTile + kMaskPad];
  __shared__ int64_t lds_off[kOffCap];
  const int tid = threadIdx.x;
  const int64_t* __restrict__ offsets = a.offsets;
  // The byte range is read on the device, so one launch shape serves any batch.
  a.lo = offsets[0];
  a.hi = offsets[a.n];
  a.c0 = a.lo - (int64_t)((reinterpret_cast<uintptr_t>(a.data) + (uintptr_t)a.lo) & 15);
  // tiles cover [c0, hi]: position hi holds the end check of the last string
  const int64_t tiles = (a.hi + 1 - a.c0 + kTile - 1) / kTile;
  const int64_t per_block = (tiles + gridDim.x - 1) / gridDim.x;
  int64_t t = (int64_t)blockIdx.x * per_block;
  const int64_t t_end = t + per_block < tiles ? t + per_block : tiles;
  if (t >= t_end) return;
  // boundaries at or after the first tile's mask window
  int64_t k0 = block_lower_bound(offsets, a.n, a.c0 + t * kTile - 4, tid);

  for (; t < t_end; ++t) {
    const int64_t ts = a.c0 + t * kTile;                   // tile start position
    const int64_t te = ts + kTile;
    // 1. string-start mask for positions [ts - 4, te)
    reinterpret_cast<uint4*>(smask)[tid] = make_uint4(0, 0, 0, 0);
    if (tid == 0) reinterpret_cast<uint4*>(smask)[256] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    int64_t cnt = 0, cnt_next = 0;
    for (;;) {
      const int64_t idx = k0 + cnt + tid;
      const int64_t v = idx <= a.n ? offsets[idx] : INT64_MAX;
      const bool in = v < te;
      if (in) {
        smask[v - ts + kMaskPad] = 0xFF;
        if (cnt + tid < kOffCap) lds_off[cnt + tid] = v;
      }
      const int c = __syncthreads_count(in);
      cnt_next += __syncthreads_count(v < te - 4);
      cnt += c;
      if (c < 256) break;
    }
    const int64_t k1 = k0 + cnt;                           // boundaries in the window: [k0, k1)
    __syncthreads();

    // 2. load the chunk and the dword before it (bytes outside [lo, hi) read as zero)
    const int64_t c = ts + (int64_t)tid * 16;
    uint4 x = make_uint4(0, 0, 0, 0);
    uint32_t p = 0;
    const bool inside = c >= a.lo && c + 16 <= a.hi;
    if (inside) {
      x = *reinterpret_cast<const uint4*>(a.data + c);
      if (c - 4 >= a.lo) p = *reinterpret_cast<const uint32_t*>(a.data + c - 4);
      else {
        for (int b = 0; b < 4; ++b) { const int64_t q = c - 4 + b; if (q >= a.lo) p |= (uint32_t)a.data[q] << (8 * b); }
      }
    } else if (c - 4 < a.hi && c + 16 > a.lo) {
      // edge chunk: its 20-byte window [c-4, c+16) overlaps [lo, hi); byte loads in range only
      uint32_t w[5] = {0, 0, 0, 0, 0};
      for (int k = 0; k < 20; ++k) {
        const int64_t q = c - 4 + k;
        if (q >= a.lo && q < a.hi) w[k >> 2] |= (uint32_t)a.data[q] << (8 * (k & 3));
      }
      p = w[0]; x = make_uint4(w[1], w[2], w[3], w[4]);
    }
    const uint4 s4 = *reinterpret_cast<const uint4*>(smask + tid * 16 + kMaskPad);
    const uint32_t sp = *reinterpret_cast<const uint32_t*>(smask + tid * 16 + kMaskPad - 4);

    // 3. checks (section 6.4 skip when the chunk, its halo and the wave are all ASCII)
    bool skip = false;
    {
      const uint32_t hi7 = (x.x | x.y | x.z | x.w | p) & 0x80808080u;
      skip = __all(hi7 == 0);
    }
    uint32_t acc = 0;
    uint32_t e[4], tl[4];
    if (!skip) {
      e[0] = masked_errors(x.x, p, s4.x, sp, &tl[0]);
      e[1] = masked_errors(x.y, x.x, s4.y, s4.x, &tl[1]);
      e[2] = masked_errors(x.z, x.y, s4.z, s4.y, &tl[2]);
      e[3] = masked_errors(x.w, x.z, s4.w, s4.z, &tl[3]);
      acc = e[0] | e[1] | e[2] | e[3] | tl[0] | tl[1] | tl[2] | tl[3];
    }
    // 4. rare: attribute errors to strings
    if (__builtin_expect(acc != 0, 0)) {
      int64_t last_k = -1;
      for (int j = 0; j < 4; ++j) {
        for (int b = 0; b < 4; ++b) {
          const int64_t pos = c + 4 * j + b;
          if ((tl[j] >> (8 * b)) & 0xFF) {
            if (pos - 1 >= a.lo && pos <= a.hi) {
              const int64_t k = string_of(pos - 1, offsets, k0, k1, lds_off);
              if (k >= 0 && k < a.n && k != last_k) {
                atomicMin(reinterpret_cast<unsigned long long*>(a.tmp + k),
                          (unsigned long long)(pos - offsets[k]));
              }
            }
          }
          if ((e[j] >> (8 * b)) & 0xFF) {
            if (pos >= a.lo && pos < a.hi) {
              const int64_t k = string_of(pos, offsets, k0, k1, lds_off);
              if (k >= 0 && k < a.n && k != last_k) {
                atomicMin(reinterpret_cast<unsigned long long*>(a.tmp + k),
                          (unsigned long long)(pos - offsets[k]));
                last_k = k;  // later positions of this string cannot be earlier
              }
            }
          }
        }
      }
    }
    // 5. next tile's window starts at te - 4
    k0 += cnt_next;
    __syncthreads();
  }
}

// Per string: first detection -> first-error offset; flags.
__global__ void batch_finalize(BatchArgs a) {
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

hipError_t launch_batch(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err,
                        const TuneBatch& cfg, int num_cus, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  BatchArgs a;
  a.data = data; a.offsets = offsets; a.n = n; a.lo = a.hi = a.c0 = 0;
  a.flags = flags; a.first_err = first_err;
  a.tmp = first_err;  // per-string detections are staged in the output array
  const int blocks = num_cus * (cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : 1);
  int fin_blocks = (int)((n + 255) / 256);
  if (fin_blocks > num_cus * 8) fin_blocks = num_cus * 8;
  hipLaunchKernelGGL(batch_init, dim3(fin_blocks), dim3(256), 0, st, a.tmp, n);
  hipLaunchKernelGGL(batch_main, dim3(blocks), dim3(256), 0, st, a);
  hipLaunchKernelGGL(batch_finalize, dim3(fin_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace utf8v
