// Diagnostic and measurement kernels: per-position classification dump, and the
// read / copy ceilings of the memory system (the GPU analogue of the paper's
// memcpy reference column in Tables 11-12).
#include "common.hpp"
#include "lookup.hpp"

namespace utf8v {

// sc[i] = classification byte (section 6.1) and err[i] = sc ^ must23 (section 6.2)
// at positions 0..n; position n is the end check on a virtual zero byte (6.3).
__global__ void classify_dump(const uint8_t* __restrict__ buf, uint64_t n, uint8_t* sc, uint8_t* err) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // dword index
  const uint64_t base = q * 4;
  if (base > n) return;
  uint32_t w[2] = {0, 0};
  for (int k = 0; k < 8; ++k) {
    const int64_t pos = (int64_t)base - 4 + k;
    if (pos >= 0 && (uint64_t)pos < n) w[k >> 2] |= (uint32_t)buf[pos] << (8 * (k & 3));
  }
  const uint32_t prev1 = align(w[1], w[0], 3), prev2 = align(w[1], w[0], 2), prev3 = align(w[1], w[0], 1);
  const uint32_t c = classify(w[1], prev1, prev2);
  const uint32_t e = c ^ must23(prev2, prev3);
  for (int b = 0; b < 4; ++b) {
    if (base + b <= n) {
      sc[base + b] = (uint8_t)(c >> (8 * b));
      err[base + b] = (uint8_t)(e >> (8 * b));
    }
  }
}

hipError_t launch_classify(const uint8_t* buf, uint64_t n, uint8_t* sc, uint8_t* err, hipStream_t st) {
  const uint64_t dwords = n / 4 + 1;
  hipLaunchKernelGGL(classify_dump, dim3((unsigned)((dwords + 255) / 256)), dim3(256), 0, st, buf, n, sc, err);
  return hipGetLastError();
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Read ceiling: every wave reads one 4 KiB tile (four 1 KiB slabs, one
// non-temporal dwordx4 per lane each) and ORs it -- the load pattern of the
// validator without its arithmetic.  Words past the last whole tile are read
// by block 0.  n is a multiple of 16.
__global__ __launch_bounds__(256) void read_or(const uint8_t* __restrict__ buf, uint64_t n, uint32_t* out) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t tiles = n / 4096;
  uint32_t acc = 0;
  if (wave < tiles) {
    const uint8_t* b = buf + wave * 4096 + lane * 16;
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(b + u * 1024));
#pragma unroll
    for (int u = 0; u < 4; ++u) acc |= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  if (blockIdx.x == 0) {
    for (uint64_t i = tiles * 4096 + (uint64_t)threadIdx.x * 16; i < n; i += 256 * 16) {
      const u32x4 v = *reinterpret_cast<const u32x4*>(buf + i);
      acc |= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  if (__any(acc != 0)) {
    for (int off = 32; off > 0; off >>= 1) acc |= __shfl_xor(acc, off);
    // only bits not yet set need the atomic (keeps a million waves off one address)
    if (lane == 0 && (acc & ~__hip_atomic_load(out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
      atomicOr(out, acc);
  }
}

// Copy ceiling: each wave moves one 4 KiB tile (four 16-byte loads per lane in flight,
// then four stores; both non-temporal), the last block also the tail past whole tiles.
__global__ __launch_bounds__(256) void copy_tiles(const uint8_t* __restrict__ s, uint8_t* __restrict__ d, uint64_t n) {
  const uint64_t tiles = n / 4096;
  const uint64_t wave = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t lane = threadIdx.x & 63;
  if (wave < tiles) {
    const uint64_t base = wave * 4096 + lane * 16;
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(s + base + u * 1024));
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], reinterpret_cast<u32x4*>(d + base + u * 1024));
  }
  if (blockIdx.x == gridDim.x - 1)
    for (uint64_t i = tiles * 4096 + (uint64_t)threadIdx.x * 16; i < n; i += 256 * 16)
      *reinterpret_cast<u32x4*>(d + i) = *reinterpret_cast<const u32x4*>(s + i);
}

hipError_t launch_read_ceiling(const uint8_t* buf, uint64_t n, uint32_t* out, int num_cus, hipStream_t st) {
  (void)num_cus;
  const uint64_t waves = n / 4096;
  const unsigned blocks = (unsigned)((waves + 3) / 4 > 0 ? (waves + 3) / 4 : 1);
  hipLaunchKernelGGL(read_or, dim3(blocks), dim3(256), 0, st, buf, n, out);
  return hipGetLastError();
}

hipError_t launch_copy(const uint8_t* src, uint8_t* dst, uint64_t n, int num_cus, hipStream_t st) {
  (void)num_cus;
  const uint64_t waves = n / 4096;
  const unsigned blocks = (unsigned)((waves + 3) / 4 > 0 ? (waves + 3) / 4 : 1);
  hipLaunchKernelGGL(copy_tiles, dim3(blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

// Which rule of section 3 the ill-formed character starting at b[s] breaks
// (b = one string of len bytes): 1 five or more header bits, 2 too short, 3 too
// long, 4 overlong, 5 too large, 6 surrogate; 0 if s is not an error position.
// Malformed sequences (1-3) rank first: only a complete sequence has a code
// point.  The code point rules are read off the lead and second byte ranges.
__device__ uint8_t class_at(const uint8_t* __restrict__ b, int64_t len, int64_t s) {
  if (s < 0 || s >= len) return 0;
  const uint32_t c = b[s];
  if (c < 0x80) return 0;
  if (c < 0xC0) return 3;
  if (c >= 0xF8) return 1;
  const int need = c >= 0xF0 ? 3 : c >= 0xE0 ? 2 : 1;  // continuation bytes the header announces
  for (int k = 1; k <= need; ++k)
    if (s + k >= len || (b[s + k] & 0xC0u) != 0x80u) return 2;
  const uint32_t b1 = b[s + 1];
  if (c <= 0xC1 || (c == 0xE0 && b1 < 0xA0) || (c == 0xF0 && b1 < 0x90)) return 4;
  if (c >= 0xF5 || (c == 0xF4 && b1 >= 0x90)) return 5;
  if (c == 0xED && b1 >= 0xA0) return 6;
  return 0;
}

__global__ void error_classes(const uint8_t* __restrict__ data, const int64_t* __restrict__ offsets, int64_t n,
                              const int64_t* __restrict__ first_err, uint8_t* __restrict__ out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = first_err[k];
    out[k] = s < 0 ? 0 : class_at(data + offsets[k], offsets[k + 1] - offsets[k], s);
  }
}

__global__ void error_class_one(const uint8_t* __restrict__ buf, int64_t len, const int64_t* __restrict__ first_err,
                                uint8_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = class_at(buf, len, *first_err);
}

hipError_t launch_error_classes(const uint8_t* data, const int64_t* offsets, int64_t n, const int64_t* first_err,
                                uint8_t* out, int num_cus, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > (int64_t)num_cus * 8) blocks = (int64_t)num_cus * 8;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(error_classes, dim3((unsigned)blocks), dim3(256), 0, st, data, offsets, n, first_err, out);
  return hipGetLastError();
}

hipError_t launch_error_class_one(const uint8_t* buf, int64_t len, const int64_t* first_err, uint8_t* out,
                                  hipStream_t st) {
  hipLaunchKernelGGL(error_class_one, dim3(1), dim3(64), 0, st, buf, len, first_err, out);
  return hipGetLastError();
}

// Stream state {first-error offset, history}: empty stream.
__global__ void stream_reset(int64_t* first_err, unsigned long long* hist) {
  if (threadIdx.x == 0) {
    *first_err = -1;
    *hist = 0ull;
  }
}

hipError_t launch_stream_reset(int64_t* first_err, unsigned long long* hist, hipStream_t st) {
  hipLaunchKernelGGL(stream_reset, dim3(1), dim3(64), 0, st, first_err, hist);
  return hipGetLastError();
}

}  // namespace utf8v
