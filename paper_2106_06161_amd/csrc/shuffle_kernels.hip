// Batch preparation kernels, workspace initialisation and the host-side
// launchers for the fused shuffle kernels (templates in shuffle_impl.h,
// instantiated per element size in inst_eb*.hip).
#include <map>
#include <utility>

#include "bshuffle.h"
#include "shuffle_impl.h"

namespace bsd {

// Batch set-up, first pass (one thread per segment, 256 segments per
// workgroup): per-segment records, domain bits and masked round keys; the
// segment's tile count; its tile offset within its workgroup's 256 segments
// (stored in first_tile for now); the workgroup's tile total and whether any
// of its segments is malformed (offsets[0] != 0, decreasing, past
// total_items, or more than 32 index bits).
__global__ __launch_bounds__(kSegmentsPerBlock) void batch_segments_kernel(const BatchArgs a) {
  __shared__ uint32_t warp_sums[kSegmentsPerBlock / 64];
  __shared__ uint32_t bad;
  const uint32_t tid = threadIdx.x;
  const uint32_t s = blockIdx.x * kSegmentsPerBlock + tid;
  if (tid == 0) bad = (blockIdx.x == 0 && a.offsets[0] != 0) ? 1u : 0u;
  __syncthreads();
  uint32_t tiles = 0;
  if (s < a.num_segments) {
    const int64_t lo = a.offsets[s], hi = a.offsets[s + 1];
    if (hi < lo || lo < 0 || uint64_t(hi) > a.total_items) {
      atomicOr(&bad, 1u);
    } else {
      const uint64_t n = uint64_t(hi - lo);
      const uint32_t k = domain_bits_dev(n);
      if (k > 32) atomicOr(&bad, 1u);
      const uint64_t dom = uint64_t(1) << min(k, 40u);
      // empty segments, and those the one-wavefront kernel takes, get no tile
      tiles = (n == 0 || k <= a.small_bits) ? 0u
                                            : uint32_t(min<uint64_t>((dom + a.tile - 1) / a.tile, 0xFFFFFFFFull));
      a.segs[s].first = uint64_t(lo);
      a.segs[s].n = n;
      a.segs[s].k = k;
      // round keys masked to the half width, then a 0 (see vp_encrypt)
      const uint32_t wmask = (1u << (k >> 1)) - 1u;
      uint32_t* keys = a.keys + uint64_t(s) * (a.rounds + 1);
      uint64_t st = a.seeds[s];
      for (uint32_t r = 0; r < a.rounds; ++r) keys[r] = uint32_t(splitmix64_next(st)) & wmask;
      keys[a.rounds] = 0;
    }
  }
  // workgroup exclusive scan of `tiles` (a segment's tiles fit 2^21, 256 of
  // them fit 32 bits)
  uint32_t v = tiles;
  const uint32_t lane = tid & 63u, warp = tid >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off, 64);
    if (lane >= uint32_t(off)) v += t;
  }
  if (lane == 63) warp_sums[warp] = v;
  __syncthreads();
  uint32_t warp_prefix = 0, block_total = 0;
#pragma unroll
  for (uint32_t w = 0; w < kSegmentsPerBlock / 64; ++w) {
    warp_prefix += (w < warp) ? warp_sums[w] : 0u;
    block_total += warp_sums[w];
  }
  if (s < a.num_segments) a.segs[s].first_tile = warp_prefix + v - tiles;
  if (tid == 0) {
    a.block_sums[blockIdx.x] = block_total;
    a.block_bad[blockIdx.x] = bad;
  }
}

// Batch set-up, second pass (one workgroup): exclusive scan of the
// workgroups' tile totals, each segment's first tile made global, the batch
// accepted or rejected (a malformed segment, or more tiles than the
// workspace holds: then no tile runs and bs_workspace_error reports
// BS_EDEVICE), and the launch's header fields.
constexpr uint32_t kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void batch_scan_kernel(const BatchArgs a) {
  __shared__ uint64_t warp_sums[kScanThreads / 64];
  __shared__ uint64_t carry;
  __shared__ uint32_t bad;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, warp = tid >> 6;
  const uint32_t blocks = (a.num_segments + kSegmentsPerBlock - 1) / kSegmentsPerBlock;
  if (tid == 0) {
    carry = 0;
    bad = 0;
  }
  __syncthreads();
  for (uint32_t base = 0; base < blocks; base += kScanThreads) {
    const uint32_t b = base + tid;
    const uint64_t c = b < blocks ? a.block_sums[b] : 0u;
    if (b < blocks && a.block_bad[b]) atomicOr(&bad, 1u);
    uint64_t v = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t t = __shfl_up(v, off, 64);
      if (lane >= uint32_t(off)) v += t;
    }
    if (lane == 63) warp_sums[warp] = v;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
      before += (w < warp) ? warp_sums[w] : 0u;
      total += warp_sums[w];
    }
    // the workgroup's exclusive prefix replaces its total (clamped: a batch
    // that large is rejected below)
    if (b < blocks) a.block_sums[b] = uint32_t(min<uint64_t>(carry + before + v - c, 0xFFFFFFFFull));
    __syncthreads();
    if (tid == 0) carry += total;
    __syncthreads();
  }
  if (tid == 0 && carry > a.capacity) bad = 1u;
  __syncthreads();
  if (!bad) {
    for (uint32_t s = tid; s < a.num_segments; s += kScanThreads)
      a.segs[s].first_tile += a.block_sums[s / kSegmentsPerBlock];
  }
  if (tid == 0) {
    const uint32_t total = bad ? 0u : uint32_t(carry);
    if (bad) atomicOr(&a.hdr->error, kErrBadBatch);
    a.hdr->batch_bad = bad;  // read by the one-wavefront kernel
    // XCD ranges start as one range (every tile on XCD 0's counter, which all
    // workgroups reach); with ranges on, batch_fill_kernel moves each boundary
    // down to the first segment that starts at or after x/8 of the tiles
    a.hdr->xcd_first[0] = 0;
    for (uint32_t x = 1; x <= kXcds; ++x) a.hdr->xcd_first[x] = total;
    __hip_atomic_store(&a.hdr->batch_tiles, total, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Marks which segment owns every tile: one wavefront per segment.
__global__ __launch_bounds__(256) void batch_fill_kernel(const BatchArgs a) {
  const uint32_t waves_total = gridDim.x * (blockDim.x / 64);
  const uint32_t wave_global = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t total = __hip_atomic_load(&a.hdr->batch_tiles, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
  if (total == 0) return;
  const bool ranges = a.xcd_mode == 1 ||
                      (a.xcd_mode == 2 && uint64_t(total) >= uint64_t(kXcdMinTilesPerSegment) * a.num_segments);
  for (uint32_t s = wave_global; s < a.num_segments; s += waves_total) {
    const SegmentInfo si = a.segs[s];
    // XCD ranges of whole segments with about total/kXcds tiles each: the
    // boundary of range x is the first segment start at or after x*total/kXcds
    // (segments without tiles share the next segment's start)
    if (ranges && lane > 0 && lane < kXcds) {
      const uint32_t p = uint32_t((uint64_t(lane) * total + kXcds - 1) / kXcds);
      const uint32_t prev = (s == 0) ? 0u : a.segs[s - 1].first_tile;
      if (si.first_tile >= p && (s == 0 || prev < p)) atomicMin(&a.hdr->xcd_first[lane], si.first_tile);
    }
    if (si.n == 0 || si.k <= a.small_bits) continue;  // no tiles
    const uint64_t dom = uint64_t(1) << si.k;
    const uint32_t tiles = uint32_t((dom + a.tile - 1) / a.tile);
    for (uint32_t t = lane; t < tiles; t += 64) a.tile_segment[si.first_tile + t] = s;
  }
}

// Zeroes a batched launch's tables once its kernels are done with them (16
// bytes per store; the region is 256-byte aligned and sized).
__global__ __launch_bounds__(256) void zero_tables_kernel(uint4* p, uint64_t count16) {
  const uint4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count16; i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = z;
}

// Zero-fills a workspace and records its status-word capacity in the header.
__global__ void zero_fill_kernel(uint32_t* p, uint64_t words, uint32_t capacity_words) {
  constexpr uint64_t kCapacityWord = offsetof(WorkspaceHeader, capacity) / sizeof(uint32_t);
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < words; i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = (i == kCapacityWord) ? capacity_words : 0u;
}

// Moves the workspace's sticky error bits into *status as a status code and
// clears them, in stream order (one thread; no host round trip).
__global__ void take_error_kernel(WorkspaceHeader* hdr, int32_t* status) {
  const uint32_t err = atomicExch(&hdr->error, 0u);
  *status = (err & kErrTimeout) ? BS_ETIMEOUT : (err & kErrBadBatch) ? BS_EDEVICE : BS_OK;
}

bool config_supported(const LaunchConfig& c) {
#define BSD_MATCH(W, I, D) \
  if (c.waves == W && c.items == I && c.depth == D) return true;
  BSD_FOR_EACH_SHAPE(BSD_MATCH)
#undef BSD_MATCH
#define BSD_MATCH(W, I) \
  if (c.waves == W && c.items == I && (c.depth == kDepthCompact || c.depth == kDepthCompactPipe)) return true;
  BSD_FOR_EACH_COMPACT_SHAPE(BSD_MATCH)
#undef BSD_MATCH
  return false;
}

// Workgroups to launch: one per tile (kGridOnePerTile), grid_mult per CU, or
// (grid_mult == 0) as many as the device keeps resident at once, so the grid
// is persistent and every workgroup loops over tickets.
static uint32_t resident_groups(const void* fn, uint32_t threads, uint32_t num_cus) {
  static std::map<std::pair<const void*, uint32_t>, uint32_t> cache;
  auto key = std::make_pair(fn, threads);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, int(threads), 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint32_t g = uint32_t(per_cu) * num_cus;
  cache[key] = g;
  return g;
}

static uint32_t grid_for(uint64_t tiles, const LaunchConfig& cfg, uint32_t num_cus, const void* fn) {
  uint64_t g = tiles;
  if (cfg.grid_mult != kGridOnePerTile) {
    const uint64_t persistent =
        cfg.grid_mult == 0 ? resident_groups(fn, cfg.waves * 64, num_cus) : uint64_t(cfg.grid_mult) * num_cus;
    if (persistent < g) g = persistent;
  }
  if (g == 0) g = 1;
  return uint32_t(g);
}

hipError_t launch_single(const SingleArgs& a0, uint32_t eb, bool nt, const LaunchConfig& cfg0, uint32_t num_cus,
                         hipStream_t stream) {
  const bool wide = a0.domain > (uint64_t(1) << 32);
  LaunchConfig cfg = cfg0;
  if (wide) cfg.waves = kWideWaves, cfg.items = kWideItems, cfg.depth = kDepthCompactPipe;
  SingleArgs a = a0;
  a.nontemporal = nt ? 1u : 0u;
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  SingleFn fn = nullptr;
  switch (eb) {
    case 0: fn = pick_single_0(odd, wide, cfg); break;
    case 1: fn = pick_single_1(odd, wide, cfg); break;
    case 2: fn = pick_single_2(odd, wide, cfg); break;
    case 4: fn = pick_single_4(odd, wide, cfg); break;
    case 8: fn = pick_single_8(odd, wide, cfg); break;
    case 16: fn = pick_single_16(odd, wide, cfg); break;
    default: return hipErrorInvalidValue;
  }
  if (!fn) return hipErrorInvalidValue;
  const uint32_t grid = grid_for(a.num_tiles, cfg, num_cus, reinterpret_cast<const void*>(fn));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * 64), 0, stream, a);
  return hipGetLastError();
}

LaunchConfig batch_config(const LaunchConfig& c) {
  return config_supported(c) ? c : LaunchConfig{16, 16, 1, c.grid_mult};
}

hipError_t launch_batched(const BatchArgs& a, uint32_t eb, const LaunchConfig& cfg, uint32_t num_cus,
                          hipStream_t stream) {
  BatchFn fn = nullptr;
  switch (eb) {
    case 1: fn = pick_batch_1(cfg); break;
    case 2: fn = pick_batch_2(cfg); break;
    case 4: fn = pick_batch_4(cfg); break;
    case 8: fn = pick_batch_8(cfg); break;
    case 16: fn = pick_batch_16(cfg); break;
    default: return hipErrorInvalidValue;
  }
  if (!fn) return hipErrorInvalidValue;
  const uint32_t seg_blocks = (a.num_segments + kSegmentsPerBlock - 1) / kSegmentsPerBlock;
  hipLaunchKernelGGL(batch_segments_kernel, dim3(seg_blocks), dim3(kSegmentsPerBlock), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t fill_blocks = std::max(1u, std::min(1024u, (a.num_segments + 3u) / 4u));
  hipLaunchKernelGGL(batch_fill_kernel, dim3(fill_blocks), dim3(256), 0, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Segments small enough for one wavefront first: up to 32 one-wavefront
  // workgroups per CU (8 per SIMD), each taking segments in a fixed stride.
  // They run before the tiled kernel because that kernel's last workgroup may
  // clear status words past this launch's own (at a tag wrap), which can
  // reach the tables.
  if (a.small_bits != 0) {
    BatchFn small = nullptr;
    switch (eb) {
      case 1: small = pick_batch_small_1(); break;
      case 2: small = pick_batch_small_2(); break;
      case 4: small = pick_batch_small_4(); break;
      case 8: small = pick_batch_small_8(); break;
      case 16: small = pick_batch_small_16(); break;
      default: return hipErrorInvalidValue;
    }
    const uint32_t small_grid = std::max(1u, std::min(a.num_segments, num_cus * 32u));
    hipLaunchKernelGGL(small, dim3(small_grid), dim3(64), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // The grid never exceeds the workspace's tile capacity; surplus workgroups
  // exit at their first ticket.
  const uint32_t grid = grid_for(a.capacity, cfg, num_cus, reinterpret_cast<const void*>(fn));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * 64), 0, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // The tables sit where a later launch with more tiles keeps status words:
  // leave them zero.
  const uint64_t count16 = a.tables_bytes / 16;
  const uint32_t zero_blocks = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(1024, (count16 + 255) / 256)));
  hipLaunchKernelGGL(zero_tables_kernel, dim3(zero_blocks), dim3(256), 0, stream, reinterpret_cast<uint4*>(a.tables),
                     count16);
  return hipGetLastError();
}

// Exclusive scan of per-tile counts (one workgroup; the tile count is small).
__global__ __launch_bounds__(1024) void tile_prefix_kernel(const uint64_t* counts, uint64_t* prefix, uint32_t tiles) {
  __shared__ uint64_t warp_sums[16];
  __shared__ uint64_t carry;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, warp = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < tiles; base += 1024) {
    const uint32_t i = base + tid;
    const uint64_t c = i < tiles ? counts[i] : 0;
    uint64_t v = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t t = __shfl_up(v, off, 64);
      if (lane >= uint32_t(off)) v += t;
    }
    if (lane == 63) warp_sums[warp] = v;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      before += (w < warp) ? warp_sums[w] : 0;
      total += warp_sums[w];
    }
    if (i < tiles) prefix[i] = carry + before + v - c;
    __syncthreads();
    if (tid == 0) carry += total;
    __syncthreads();
  }
}

// f(i) for every i of the padded domain (the unfused variant's first pass).
template <bool ODD>
__global__ __launch_bounds__(256) void cipher_table_kernel(const SingleArgs a, uint32_t* table) {
  constexpr int kItems = 8;
  const uint64_t stride = uint64_t(gridDim.x) * 256 * kItems;
  for (uint64_t base = uint64_t(blockIdx.x) * 256 * kItems + threadIdx.x; base < a.domain; base += stride) {
    uint32_t L[kItems], R[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t x = uint32_t(base + uint64_t(j) * 256);
      L[j] = (x >> a.cs.r) & (a.cs.wmask & 0xFFFFFFu);
      R[j] = x;
    }
    vp_encrypt<ODD, kItems>(L, R, a.cs, a.rounds, a.key);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t x = base + uint64_t(j) * 256;
      if (x < a.domain) table[x] = (L[j] << a.cs.r) | (R[j] & a.cs.rmask);
    }
  }
}

hipError_t launch_workspace_init(void* ws, size_t bytes, hipStream_t stream) {
  const uint64_t words = bytes / 4;
  const uint64_t cap = bytes > sizeof(WorkspaceHeader) ? (bytes - sizeof(WorkspaceHeader)) / 8 : 0;
  const uint32_t blocks = uint32_t(std::min<uint64_t>(1024, (words + 255) / 256 + 1));
  hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(ws), words,
                     uint32_t(std::min<uint64_t>(cap, 0xFFFFFFFFull)));
  return hipGetLastError();
}

hipError_t launch_take_error(void* ws, int32_t* status, hipStream_t stream) {
  hipLaunchKernelGGL(take_error_kernel, dim3(1), dim3(1), 0, stream, static_cast<WorkspaceHeader*>(ws), status);
  return hipGetLastError();
}

hipError_t launch_variant(const SingleArgs& a, uint32_t variant, uint32_t eb, uint32_t num_cus, hipStream_t stream) {
  const bool wide = a.domain > (uint64_t(1) << 32);
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  SingleFn fn = nullptr;
  switch (eb) {
    case 1: fn = pick_variant_1(variant, odd, wide); break;
    case 2: fn = pick_variant_2(variant, odd, wide); break;
    case 4: fn = pick_variant_4(variant, odd, wide); break;
    case 8: fn = pick_variant_8(variant, odd, wide); break;
    case 16: fn = pick_variant_16(variant, odd, wide); break;
    default: return hipErrorInvalidValue;
  }
  if (!fn) return hipErrorInvalidValue;
  LaunchConfig cfg = {wide ? kWideWaves : uint32_t(kAltWaves), wide ? kWideItems : uint32_t(kAltItems), 1, 0};
  const uint32_t grid = grid_for(a.num_tiles, cfg, num_cus, reinterpret_cast<const void*>(fn));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(cfg.waves * 64), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_tile_counts(const SingleArgs& a, hipStream_t stream) {
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  const uint32_t grid = std::max(1u, std::min(a.num_tiles, 4096u));
  if (odd)
    hipLaunchKernelGGL((tile_count_kernel<true, kAltWaves, kAltItems>), dim3(grid), dim3(kAltWaves * 64), 0, stream, a);
  else
    hipLaunchKernelGGL((tile_count_kernel<false, kAltWaves, kAltItems>), dim3(grid), dim3(kAltWaves * 64), 0, stream,
                       a);
  return hipGetLastError();
}

hipError_t launch_tile_prefix(const uint64_t* counts, uint64_t* prefix, uint32_t tiles, hipStream_t stream) {
  hipLaunchKernelGGL(tile_prefix_kernel, dim3(1), dim3(1024), 0, stream, counts, prefix, tiles);
  return hipGetLastError();
}

hipError_t launch_cipher_table(const SingleArgs& a, uint32_t* table, hipStream_t stream) {
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  const uint64_t want = (a.domain + 256 * 8 - 1) / (256 * 8);
  const uint32_t grid = uint32_t(std::min<uint64_t>(want, 65536));
  if (odd)
    hipLaunchKernelGGL(cipher_table_kernel<true>, dim3(grid), dim3(256), 0, stream, a, table);
  else
    hipLaunchKernelGGL(cipher_table_kernel<false>, dim3(grid), dim3(256), 0, stream, a, table);
  return hipGetLastError();
}

}  // namespace bsd
