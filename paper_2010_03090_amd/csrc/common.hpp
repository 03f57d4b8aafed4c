// Shared definitions of the gfx950 validator library (kernels and host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utf8v {

constexpr uint64_t kNone = ~uint64_t(0);          // "no error detected" for 64-bit positions
constexpr int64_t kNoneRel = INT64_MAX;           // same, for per-string relative offsets
constexpr int kDppWaveRor1 = 0x13C;               // DPP wave_ror:1 -- lane l reads lane (l-1) mod 64

struct TuneSingle {
  int unroll = 4;             // dwordx4 loads in flight per lane (1 KiB per wave each)
  int waves_per_cu = 24;      // persistent waves per compute unit (large = one tile per wave)
  int min_tiles_per_wave = 1;
  int ascii = 1;              // section 6.4 fast path for all-ASCII slabs
};

struct TuneBatch {
  int waves_per_cu = 16;      // persistent grid: one-wave workgroups per compute unit
  int ascii = 1;
};

struct SingleArgs {
  const uint8_t* buf;
  uint64_t i0, i1;            // interior [i0, i1): 16-byte aligned
  uint64_t tiles, tiles_per_wave;
  unsigned long long* dmin;
};

struct FinalizeArgs {
  const uint8_t* buf;
  uint64_t n, i0, i1;
  unsigned long long* dmin;
  int64_t* out;
};

struct BatchArgs {
  const uint8_t* data;
  const int64_t* offsets;
  int64_t n;                  // strings
  unsigned long long* slot;   // workspace, one word per wave: arrivals and partial first detection
  uint8_t* flags;
  int64_t* first_err;
};

// Wave minimum of v (kNone = none), then one atomicMin into *dst unless *dst is
// already lower (on inputs with errors everywhere, most waves then skip the atomic).
__device__ __forceinline__ void wave_min_to(unsigned long long* dst, uint64_t v, int lane) {
  if (__any(v != kNone)) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor((unsigned long long)v, off);
      v = o < v ? o : v;
    }
    if (lane == 0 && v < __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMin(dst, (unsigned long long)v);
  }
}

hipError_t launch_single(const uint8_t* buf, uint64_t n, unsigned long long* dmin, int64_t* out,
                         const TuneSingle& cfg, int num_cus, hipStream_t st);
BatchArgs batch_args(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err,
                     unsigned long long* slot);
hipError_t launch_batch(const BatchArgs& a, const TuneBatch& cfg, int num_cus, hipStream_t st);
hipError_t launch_batch_slots_init(unsigned long long* slot, int slots, hipStream_t st);
hipError_t capture_batch_graph(const BatchArgs* dparams, const TuneBatch& cfg, int num_cus, hipGraphExec_t* exec);
hipError_t launch_offsets_check(const int64_t* offsets, int64_t n, int* bad, int num_cus, hipStream_t st);
hipError_t launch_classify(const uint8_t* buf, uint64_t n, uint8_t* sc, uint8_t* err, hipStream_t st);
hipError_t launch_read_ceiling(const uint8_t* buf, uint64_t n, uint32_t* out, int num_cus, hipStream_t st);
hipError_t launch_copy(const uint8_t* src, uint8_t* dst, uint64_t n, int num_cus, hipStream_t st);

}  // namespace utf8v
