// Shared definitions of the gfx950 validator library (kernels and host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <limits>

namespace utf8v {

constexpr uint64_t kNone = ~uint64_t(0);          // "no error detected" for 64-bit positions
constexpr int64_t kNoneRel = INT64_MAX;           // same, for per-string relative offsets
constexpr int kDppWaveRor1 = 0x13C;               // DPP wave_ror:1 -- lane l reads lane (l-1) mod 64
constexpr int kDppWaveShr1 = 0x138;               // DPP wave_shr:1 -- lane l reads lane l-1 (l >= 1)

struct TuneSingle {
  int unroll = 4;             // dwordx4 loads in flight per lane (1 KiB per wave each)
  int waves_per_cu = 20;      // persistent waves per compute unit (large = one tile per wave)
  int min_tiles_per_wave = 1;
  int ascii = 1;              // section 6.4 fast path for all-ASCII slabs
};

struct TuneBatch {
  int waves_per_cu = 16;      // persistent grid: one-wave workgroups per compute unit
  int ascii = 1;              // section 6.4 test of all-ASCII tiles (with its back-off)
  int unroll = 4;             // 1 KiB slabs per wave tile: 4 or 8
};

// State word of a single-buffer call: arrivals << kStateShift | least detection
// position (kPosNone = none).  Idle (no arrivals, no detection) between calls.
constexpr int kStateShift = 40;
constexpr uint64_t kPosNone = (1ull << kStateShift) - 1;
constexpr int kStateGroups = 64;   // group words under the top word
constexpr int kStateStride = 32;   // words between state words (256 bytes)
constexpr int kStateWords = kStateStride * (1 + kStateGroups);

// Strings per batch: the batch kernel counts string indices in 32 bits.
constexpr int64_t kMaxBatchStrings = (int64_t(1) << 31) - 65;

struct BatchArgs {
  const uint8_t* data;
  const int64_t* offsets;
  int64_t n;                  // strings
  unsigned long long* slot;   // workspace, one word per wave: arrivals and partial first detection
  uint8_t* flags;
  int64_t* first_err;
};

hipError_t launch_single(const uint8_t* buf, uint64_t n, unsigned long long* state, int64_t* out,
                         const TuneSingle& cfg, int num_cus, hipStream_t st);
// One chunk of a stream: history = the 8 bytes before it (updated in place), base =
// its stream position; without the end check, positions past the chunk do not exist.
hipError_t launch_stream_chunk(const uint8_t* buf, uint64_t n, unsigned long long* state, int64_t* out,
                               unsigned long long* hist, int64_t base, bool end_check, bool keep_first,
                               const TuneSingle& cfg, int num_cus, hipStream_t st);
// Copy src to dst (same address modulo 16, no overlap) and validate it in the same pass.
hipError_t launch_copy_validate(uint8_t* dst, const uint8_t* src, uint64_t n, unsigned long long* state,
                                int64_t* out, const TuneSingle& cfg, int num_cus, hipStream_t st);
hipError_t launch_single_any(const uint8_t* buf, uint8_t* dst, uint64_t n, unsigned long long* state, int64_t* out,
                             unsigned long long* hist, int64_t base, bool end_check, bool keep_first,
                             const TuneSingle& cfg, int num_cus, hipStream_t st);
BatchArgs batch_args(const uint8_t* data, const int64_t* offsets, int64_t n, uint8_t* flags, int64_t* first_err,
                     unsigned long long* slot);
hipError_t launch_batch(const BatchArgs& a, const TuneBatch& cfg, int num_cus, hipStream_t st);
hipError_t launch_batch_slots_init(unsigned long long* slot, int slots, hipStream_t st);
void batch_launch_queries();   // one-time queries of the batch launch, made outside any stream capture
void single_launch_queries();  // the same for the single-buffer launches
// A one-node graph of the batch launch (num_cus, cfg fixed), and the update of its
// arguments before each replay.
hipError_t make_batch_graph(const TuneBatch& cfg, int num_cus, hipGraph_t* graph, hipGraphExec_t* exec,
                            hipGraphNode_t* node);
hipError_t set_batch_graph_args(hipGraphExec_t exec, hipGraphNode_t node, const BatchArgs& a, const TuneBatch& cfg,
                                int num_cus);
hipError_t launch_offsets_check(const int64_t* offsets, int64_t n, int* bad, int num_cus, hipStream_t st);
hipError_t launch_classify(const uint8_t* buf, uint64_t n, uint8_t* sc, uint8_t* err, hipStream_t st);
hipError_t launch_read_ceiling(const uint8_t* buf, uint64_t n, uint32_t* out, int num_cus, hipStream_t st);
hipError_t launch_copy(const uint8_t* src, uint8_t* dst, uint64_t n, int num_cus, hipStream_t st);
hipError_t launch_stream_reset(int64_t* first_err, unsigned long long* hist, hipStream_t st);
hipError_t launch_error_classes(const uint8_t* data, const int64_t* offsets, int64_t n, const int64_t* first_err,
                                uint8_t* out, int num_cus, hipStream_t st);
hipError_t launch_error_class_one(const uint8_t* buf, int64_t len, const int64_t* first_err, uint8_t* out,
                                  hipStream_t st);

// A SIMD issues from its oldest ready wave first.  In a loop bound by instruction
// issue the oldest of a SIMD's waves then runs ahead, the youngest lags, and it
// finishes its last tiles nearly alone.  When every wave of the grid is resident at
// once, the kernels lower a wave's priority as it gets through its tiles (3 for the
// first quarter, then 2, 1, 0), so the waves of a SIMD keep pace with each other and
// finish together.  (With more waves than fit, a wave that starts late would take the
// SIMD from the waves finishing before it, so the levels are left off.)
__device__ __forceinline__ void set_priority(int p) {
  switch (p) {  // s_setprio takes an immediate
    case 3: __builtin_amdgcn_s_setprio(3); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
  }
}

// The priority levels of a run of `count` tiles from tile `first`: level 3 - k from the
// tile ceil(k * count / 4) tiles into the run.  Wave-uniform; step() at each tile.  I is
// the tile index type (a 32-bit index keeps the comparisons scalar).
template <class I>
struct PriorityLevelsT {
  I first, count, next;
  int prio = 3;
  bool on;
  __device__ PriorityLevelsT(bool level, I first_tile, I tiles)
      : first(first_tile), count(tiles), next(first_tile + (tiles + 3) / 4), on(level) {
    if (on) set_priority(3);
  }
  __device__ __forceinline__ void step(I t) {
    if (!on || t < next) return;
    do {
      --prio;
      next = prio > 0 ? first + ((4 - prio) * count + 3) / 4 : std::numeric_limits<I>::max();
    } while (t >= next);
    set_priority(prio);
  }
};
using PriorityLevels = PriorityLevelsT<int64_t>;

}  // namespace utf8v
