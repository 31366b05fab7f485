// Workspace layout, tile status words and the decoupled look-back (device code).
//
// Algorithm 1 (Sec. 4) needs, for every kept padded index, the number of kept
// indices before it.  The padded domain is cut into tiles; a workgroup counts
// its tile's kept indices with wavefront ballots and an LDS scan, then finds
// the count of everything before the tile with the single-pass decoupled
// look-back (Merrill and Garland) that the paper's fully fused variant uses
// (Sec. 4, Sec. 6 "Bijective2"): every tile publishes its own count
// ("aggregate") as soon as it knows it, and its running total ("inclusive
// prefix") once it has one; a tile sums predecessors' aggregates backwards
// until it meets an inclusive prefix.  The flags never leave the chip.
//
// Status word (64 bits, written and read with single agent-scope atomics so
// that flag and value always travel together across the 8 XCD L2 caches):
//   bits 63..40  tag: low 24 bits of the workspace launch generation
//   bits 39..38  flag: 0 = nothing yet, 1 = aggregate, 2 = inclusive prefix
//   bits 37..0   value
// A word whose tag differs from the current launch's is "nothing yet", so the
// status array never needs clearing between launches; when the 24-bit tag
// wraps, the launch's last workgroup clears every status word any launch on
// the workspace has used (the header's high-water mark).  The status array
// must never hold anything but status words or zeros: batched launches keep
// their tables after their own status words and zero them once the launch is
// done, so a later launch with a larger status array cannot read stale table
// bytes as status words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsd {

constexpr uint32_t kTagBits = 24;
constexpr uint32_t kTagMask = (1u << kTagBits) - 1;
constexpr uint32_t kValueBits = 38;
constexpr uint64_t kValueMask = (uint64_t(1) << kValueBits) - 1;
constexpr uint64_t kFlagAggregate = uint64_t(1) << kValueBits;
constexpr uint64_t kFlagPrefix = uint64_t(2) << kValueBits;
constexpr uint32_t kSpinLimit = 1u << 22;  // ~seconds of polling before giving up (default)

// Look-back watchdog of a launch: polls before a wait gives up (it then sets
// the sticky timeout error and treats the nearest tile as a prefix of 0, so
// the launch still finishes), and a test hook: with stall_first set, the
// first tile of every shuffle withholds its status word, so the next tile's
// wait deterministically runs into the limit.
struct Watchdog {
  uint32_t spin_limit;
  uint32_t stall_first;
};

// Sticky device-side error bits kept in the workspace header.
constexpr uint32_t kErrTimeout = 1u;
constexpr uint32_t kErrBadBatch = 2u;

// XCDs (accelerator complex dies, one L2 each) of the device.  Workgroups are
// dispatched to them round-robin, so workgroup b runs on XCD b % kXcds.
constexpr uint32_t kXcds = 8;

// First 256 bytes of every workspace.
struct WorkspaceHeader {
  uint32_t ticket;         // next tile handed out in this launch (single shuffles)
  uint32_t done;           // workgroups finished in this launch
  uint32_t gen;            // launch generation; its low 24 bits tag status words
  uint32_t error;          // sticky error bits
  uint32_t capacity;       // status words the workspace holds (set at init; informational)
  uint32_t batch_tiles;    // batched launches: tiles of the current batch
  uint32_t xcd_ticket[kXcds];     // batched launches: next tile of each XCD's range
  uint32_t xcd_first[kXcds + 1];  // batched launches: XCD x owns tiles [xcd_first[x], xcd_first[x+1])
  uint32_t batch_bad;      // batched launches: 1 when the current batch was rejected
  uint32_t status_hwm;     // status words used by any launch since init (cleared at a tag wrap)
  uint32_t pad[39];
};
static_assert(sizeof(WorkspaceHeader) == 256, "header is 256 bytes");

__device__ __forceinline__ uint64_t status_word(uint32_t tag, uint64_t flag, uint64_t value) {
  return (uint64_t(tag) << 40) | flag | value;
}
__device__ __forceinline__ uint64_t atomic_load_agent(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Called by all 64 lanes of ONE wavefront.  `tile` indexes `status` (the
// words of the tile's own segment start at first_tile).  Publishes the tile's
// aggregate, looks back, publishes the inclusive prefix, and returns the
// exclusive prefix (kept indices before the tile, within its segment).
__device__ __forceinline__ uint64_t lookback_exclusive_prefix(uint64_t* status, uint32_t first_tile,
                                                              uint32_t tile, uint32_t tag, uint64_t aggregate,
                                                              uint32_t* error_word, Watchdog wd) {
  const uint32_t lane = lane_id();
  if (tile == first_tile) {
    if (lane == 0 && !wd.stall_first) atomic_store_agent(status + tile, status_word(tag, kFlagPrefix, aggregate));
    return 0;
  }
  if (lane == 0) atomic_store_agent(status + tile, status_word(tag, kFlagAggregate, aggregate));

  uint64_t exclusive = 0;
  int64_t window_end = int64_t(tile) - 1;  // lane l looks at tile window_end - l
  uint32_t spins = 0;
  for (;;) {
    const int64_t idx = window_end - int64_t(lane);
    const bool before_segment = idx < int64_t(first_tile);
    uint64_t word = 0;
    uint32_t flag = 0;
    uint64_t ready_mask, prefix_mask;
    for (;;) {
      if (before_segment) {
        flag = 2;  // tiles before the segment act as an inclusive prefix of 0
        word = 0;
      } else {
        word = atomic_load_agent(status + idx);
        const uint32_t wtag = uint32_t(word >> 40);
        flag = (wtag == tag) ? uint32_t((word >> kValueBits) & 3u) : 0u;
      }
      ready_mask = __ballot(flag != 0);
      prefix_mask = __ballot(flag == 2);
      // Need every lane up to the nearest inclusive prefix (or the whole window
      // when there is none) to be ready.
      const uint64_t not_ready = ~ready_mask;
      const uint64_t upto = prefix_mask ? (prefix_mask & (~prefix_mask + 1)) : 0;  // lowest P lane bit
      const uint64_t needed = upto ? ((upto << 1) - 1) : ~uint64_t(0);
      if ((not_ready & needed) == 0) break;
      if (++spins > wd.spin_limit) {
        if (lane == 0) atomicOr(error_word, kErrTimeout);
        ready_mask = ~uint64_t(0);
        prefix_mask = uint64_t(1);  // give up: treat the nearest tile as a prefix
        flag = (lane == 0) ? 2u : 0u;
        word = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (prefix_mask) {
      const uint32_t p = uint32_t(__builtin_ctzll(prefix_mask));
      // lanes below p contribute aggregates (each <= tile size), lane p its prefix
      const uint32_t agg = (lane < p) ? uint32_t(word & kValueMask) : 0u;
      const uint64_t pref_word = __shfl(word, int(p), 64);
      exclusive += uint64_t(wave_sum_u32(agg)) + (pref_word & kValueMask);
      break;
    }
    exclusive += uint64_t(wave_sum_u32(uint32_t(word & kValueMask)));
    window_end -= 64;
  }
  if (lane == 0) atomic_store_agent(status + tile, status_word(tag, kFlagPrefix, exclusive + aggregate));
  return exclusive;
}

}  // namespace bsd
