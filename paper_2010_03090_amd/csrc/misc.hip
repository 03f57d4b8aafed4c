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

// Read ceiling: OR of all 16-byte words of a 16-byte aligned buffer (n multiple of 16).
__global__ __launch_bounds__(256) void read_or(const uint4* __restrict__ p, uint64_t words, uint32_t* out) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < words; i += 4 * stride) {
    const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
    acc |= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < words; i += stride) { const uint4 a = p[i]; acc |= a.x ^ a.y ^ a.z ^ a.w; }
  if (__any(acc != 0)) {
    for (int off = 32; off > 0; off >>= 1) acc |= __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0 && acc) atomicOr(out, acc);
  }
}

__global__ __launch_bounds__(256) void copy16(const uint4* __restrict__ s, uint4* __restrict__ d, uint64_t words) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) d[i] = s[i];
}

hipError_t launch_read_ceiling(const uint8_t* buf, uint64_t n, uint32_t* out, int num_cus, hipStream_t st) {
  hipLaunchKernelGGL(read_or, dim3((unsigned)(num_cus * 8)), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(buf), n / 16, out);
  return hipGetLastError();
}

hipError_t launch_copy(const uint8_t* src, uint8_t* dst, uint64_t n, int num_cus, hipStream_t st) {
  hipLaunchKernelGGL(copy16, dim3((unsigned)(num_cus * 8)), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n / 16);
  return hipGetLastError();
}

}  // namespace utf8v
