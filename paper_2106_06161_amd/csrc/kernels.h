// Kernel argument blocks and host-side launchers shared by the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tile_scan.h"
#include "vphilox_round.h"

namespace bsd {

constexpr uint32_t kMaxRounds = 64;

// One bijective shuffle (Algorithm 1) over a padded domain of 2^k indices.
struct SingleArgs {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;          // items kept (input length)
  uint64_t domain;     // 2^k
  CipherShape cs;
  uint32_t rounds;
  uint32_t num_tiles;  // ceil(domain / tile)
  uint32_t capacity;   // status words the workspace holds
  uint32_t nontemporal;  // 1: output stores bypass cache retention
  Watchdog wd;           // look-back spin limit (and the stall test hook)
  WorkspaceHeader* hdr;
  uint64_t* status;
  const uint32_t* table;        // unfused variant: f over the padded domain
  const uint64_t* tile_prefix;  // two-pass variant: exclusive prefix of every tile
  uint64_t* tile_counts;        // two-pass variant: kept count of every tile
  uint64_t lcg_a, lcg_c;        // LCG variant: multiplier (odd) and increment, both < 2^k
  uint32_t key[kMaxRounds + 1];  // round keys masked to the half width, then 0
};

// Per-segment record written by the batch preparation kernel.
struct SegmentInfo {
  uint64_t first;       // first record of the segment in in/out
  uint64_t n;           // records in the segment
  uint32_t first_tile;  // index of the segment's first tile (and status word)
  uint32_t k;           // domain bits of the segment
};

struct BatchArgs {
  const uint8_t* in;
  uint8_t* out;
  const int64_t* offsets;  // device, num_segments + 1
  const uint64_t* seeds;   // device, num_segments
  uint64_t total_items;     // records in in/out; every offset must be <= this
  uint32_t num_segments;
  uint32_t rounds;
  uint32_t capacity;        // status words the workspace holds (= max tiles)
  uint32_t tile;            // indices per tile of the launch configuration
  uint32_t nontemporal;     // 1: output stores bypass cache retention
  Watchdog wd;              // look-back spin limit (and the stall test hook)
  uint32_t xcd_mode;        // tile ranges per XCD: 0 off, 1 on, 2 when segments average
                            // at least kXcdMinTilesPerSegment tiles
  uint32_t small_bits;      // segments of at most 2^small_bits padded indices go to the
                            // one-wavefront kernel instead of tiles (0: none)
  WorkspaceHeader* hdr;
  uint64_t* status;
  SegmentInfo* segs;        // num_segments records
  uint32_t* keys;           // num_segments * (rounds + 1): masked keys, then 0
  uint32_t* tile_segment;   // capacity entries: segment owning each tile
  uint32_t* block_sums;     // per 256 segments: tiles, then their exclusive prefix
  uint32_t* block_bad;      // per 256 segments: 1 if one of them is malformed
  uint8_t* tables;          // first byte of the tables above (256-byte aligned)
  uint64_t tables_bytes;    // bytes of all the tables (a multiple of 256), zeroed after the launch
};

constexpr uint32_t kXcdMinTilesPerSegment = 4;
constexpr uint32_t kSegmentsPerBlock = 256;  // batch set-up: segments per workgroup
// Segments whose padded domain fits one wavefront's items (64 lanes x 16)
// are shuffled by one wavefront each, with no tile, scan or look-back.
constexpr uint32_t kSmallSegmentItems = 16;
constexpr uint32_t kSmallSegmentBits = 10;  // 2^10 = 64 x kSmallSegmentItems

// Un-shuffle through f^-1 (gather form): a rank table over the padded domain,
// then out[p] = in[rank(f^-1(p))] for every p < n.
constexpr uint32_t kRankGroup = 32;                         // indices per table entry
constexpr uint32_t kRankThreads = 256;                      // entries per rank tile
constexpr uint32_t kRankTile = kRankGroup * kRankThreads;  // indices per rank tile
struct InverseArgs {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;
  uint64_t domain;        // 2^k
  CipherShape cs;
  uint32_t rounds;
  uint32_t num_tiles;     // ceil(domain / kRankTile)
  uint64_t* table;        // ceil(domain / kRankGroup) entries: kept flags (low word),
                          // kept indices before the entry within its rank tile (high word)
  uint64_t* tile_counts;  // kept indices per rank tile
  uint64_t* tile_prefix;  // exclusive prefix of tile_counts
  uint32_t key[kMaxRounds + 1];  // round keys masked to the half width, then 0
};

// The bijection alone, elementwise on 64-bit values (bs_bijection).
struct BijectionArgs {
  const uint64_t* in;
  uint64_t* out;
  uint64_t count;
  CipherShape cs;
  uint32_t rounds;
  uint32_t inverse;  // 1: apply f^-1
  uint32_t key[kMaxRounds + 1];  // round keys masked to the half width, then 0
};

// Staged form (streaming passes; see staged.hip): bucket arrays in the
// caller's scratch.  Pass-1 buckets: 2^b1 regions of 2^(k - b1) entries;
// windows: 2^(b1 + b2) regions of 2^s entries; each entry is a padded index
// (idx) and a record (val), in two arrays.
struct StagedArgs {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;
  CipherShape cs;
  uint32_t k;       // domain bits
  uint32_t rounds;
  uint32_t s;       // window bits
  uint32_t b1, b2;  // digit bits of the first and second distribution passes (b2 = 0: one pass)
  uint32_t* idx_a;   // bucket entries' padded indices (4-byte records: (index, record) pairs over idx_a and val_a)
  uint8_t* val_a;
  uint32_t* cnt_a;   // 2^b1 bucket counts
  uint16_t* idx_b;   // low 16 bits of the padded index (the place pass needs i mod 2^s, s <= 16)
  uint8_t* val_b;
  uint32_t* cnt_b;   // 2^(b1 + b2) window counts
  uint32_t* base_b;  // exclusive prefix of cnt_b
  uint32_t key[kMaxRounds + 1];  // round keys masked to the half width, then 0
};

struct LaunchConfig {
  uint32_t waves;      // wavefronts per workgroup
  uint32_t items;      // indices per lane per tile
  uint32_t depth;      // tile schedule: 1 or 2 tiles in flight with the kept records in
                       // registers, or kDepthCompact / kDepthCompactPipe (kept images
                       // compacted through LDS)
  uint32_t grid_mult;  // 0: as many workgroups as stay resident (persistent);
                       // 1..64: that many per CU; kGridOnePerTile: one per tile
};
constexpr uint32_t kGridOnePerTile = 1000;
constexpr uint32_t kDepthCompact = 8;      // kept images compacted through LDS
constexpr uint32_t kDepthCompactPipe = 9;  // same, next tile's cipher overlapping the gathers

hipError_t launch_single(const SingleArgs& a, uint32_t elem_bytes, bool nontemporal, const LaunchConfig& cfg,
                         uint32_t num_cus, hipStream_t stream);
hipError_t launch_batched(const BatchArgs& a, uint32_t elem_bytes, const LaunchConfig& cfg, uint32_t num_cus,
                          hipStream_t stream);
hipError_t launch_workspace_init(void* ws, size_t bytes, hipStream_t stream);
hipError_t launch_take_error(void* ws, int32_t* status, hipStream_t stream);
hipError_t launch_variant(const SingleArgs& a, uint32_t variant, uint32_t elem_bytes, uint32_t num_cus,
                          hipStream_t stream);
hipError_t launch_tile_counts(const SingleArgs& a, hipStream_t stream);
hipError_t launch_tile_prefix(const uint64_t* counts, uint64_t* prefix, uint32_t tiles, hipStream_t stream);
hipError_t launch_cipher_table(const SingleArgs& a, uint32_t* table, hipStream_t stream);
hipError_t launch_bijection(const BijectionArgs& a, hipStream_t stream);
hipError_t launch_unshuffle_inverse(const InverseArgs& a, uint32_t elem_bytes, hipStream_t stream);
uint32_t staged_window_bits(uint32_t elem_bytes);
bool staged_digits(uint32_t k, uint32_t elem_bytes, uint32_t* s, uint32_t* b1, uint32_t* b2);
hipError_t launch_staged(const StagedArgs& a, uint32_t elem_bytes, uint32_t num_cus, hipStream_t stream);
// The staged un-shuffle: the staged form's passes keyed by the output
// position f(i) of every kept padded index, with the record read at rank(i).
// keys: max(2^k, tile) words; tile_cnt, tile_base: one word per tile of
// unshuffle_key_tile(elem_bytes) padded indices.
uint32_t unshuffle_key_tile(uint32_t elem_bytes);
hipError_t launch_unshuffle_staged(const StagedArgs& a, uint32_t* keys, uint32_t* tile_cnt, uint32_t* tile_base,
                                   uint32_t elem_bytes, uint32_t num_cus, hipStream_t stream);

bool config_supported(const LaunchConfig& cfg);
// The shape a batched launch runs: cfg when compiled, else the default
// register shape.  The tile size follows the returned shape.
LaunchConfig batch_config(const LaunchConfig& cfg);

using SingleFn = void (*)(SingleArgs);
using BatchFn = void (*)(BatchArgs);

// Per-element-size kernel selection (one translation unit each).
// Tile shapes that are compiled: (waves per workgroup, indices per lane, depth).
#define BSD_FOR_EACH_SHAPE(X) \
  X(4, 16, 2) X(8, 16, 2) X(8, 16, 1) X(16, 16, 1) X(16, 8, 1) X(8, 8, 2) X(4, 16, 1) X(16, 16, 2) X(16, 8, 2)
// Shapes of the LDS-compacted schedule (single shuffles with k <= 32, and
// batched launches): (waves, items).
#define BSD_FOR_EACH_COMPACT_SHAPE(X) X(16, 16) X(8, 16) X(16, 8) X(8, 8) X(4, 16)
// Shape used when the index space needs 64 bits (k > 32): the pipelined
// compacted schedule for shuffles, the register schedule for the variants.
constexpr uint32_t kWideWaves = 16, kWideItems = 8;

// Kernel variants (fixed tile shape 16 waves x 16 items): what a kept index
// produces (0 gather, 1 index, 2 scatter), and how the tile prefix is found.
enum Variant : uint32_t {
  kVarIndices = 1,   // out[rank] = f(i)               (bs_permutation)
  kVarScatter = 2,   // out[f(i)] = in[rank]           (bs_unshuffle)
  kVarTwoPass = 3,   // gather, tile prefixes from a separate scan pass
  kVarFromTable = 4,  // compaction of a precomputed f table into indices
  kVarLcg = 5         // gather with the LCG as the bijection      (bs_shuffle_lcg)
};
constexpr uint32_t kAltTile = 16u * 64u * 16u;

#define BSD_DECLARE_PICK(EB)                                                    \
  SingleFn pick_single_##EB(bool odd, bool wide, const LaunchConfig& c);        \
  BatchFn pick_batch_##EB(const LaunchConfig& c);                               \
  BatchFn pick_batch_small_##EB();                                              \
  SingleFn pick_variant_##EB(uint32_t variant, bool odd, bool wide);
BSD_DECLARE_PICK(0)
BSD_DECLARE_PICK(1)
BSD_DECLARE_PICK(2)
BSD_DECLARE_PICK(4)
BSD_DECLARE_PICK(8)
BSD_DECLARE_PICK(16)
#undef BSD_DECLARE_PICK

}  // namespace bsd
