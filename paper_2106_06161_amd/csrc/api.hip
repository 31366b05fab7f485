// C ABI of libbshuffle.so: argument checks, the key schedule, workspace
// management and kernel dispatch.  Declarations and contracts are in
// include/bshuffle.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <iterator>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "bshuffle.h"
#include "bshuffle_probe.h"
#include "config_state.h"
#include "kernels.h"

static_assert(BS_GRID_ONE_PER_TILE == bsd::kGridOnePerTile, "grid constant of the ABI");

// Workspace of bs_shuffle_noalloc: a device array of static storage, one per
// GPU, held until the process ends; every bs_shuffle_noalloc call on a GPU
// uses that GPU's copy (never allocated or freed by the library).
static __device__ __align__(256) uint8_t scratch[BS_NOALLOC_SCRATCH_BYTES];
static_assert(BS_DEPTH_COMPACT == bsd::kDepthCompact, "schedule constant of the ABI");
static_assert(BS_DEPTH_COMPACT_PIPE == bsd::kDepthCompactPipe, "schedule constant of the ABI");

namespace {

thread_local int32_t g_last_hip_error = 0;

bs_status hip_fail(hipError_t e) {
  g_last_hip_error = static_cast<int32_t>(e);
  return BS_EHIP;
}

// The smallest tile any launch configuration uses: sizes the status array.
constexpr uint64_t kMinTile = 2048;  // indices; no compiled shape has a smaller tile
constexpr uint32_t kStaticMaxDomainBits = 30;  // bs_shuffle_noalloc: domains up to 2^30 (n <= 2^30)
constexpr size_t kHeaderBytes = sizeof(bsd::WorkspaceHeader);

std::mutex g_mu;
bsd::LaunchConfig g_default_cfg = {16, 16, 1, 0};
bsd::LaunchConfig g_cfg = g_default_cfg;
bool g_forced = false;  // bs_set_config with a shape: ignore the tuned table

// Tuned launch shapes keyed by (call kind, element bytes, size class).
// Single calls use the domain bits k; batched calls the bits of the mean
// segment size.
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, bsd::LaunchConfig> g_tuned;

// The tuned entry of the size class, else of the nearest tuned class of the
// same call kind and element size (the largest below, then the smallest
// above), else the default shape.
bsd::LaunchConfig pick_config(uint32_t kind, uint32_t elem_bytes, uint32_t bits) {
  if (g_forced) return g_cfg;
  auto it = g_tuned.upper_bound(std::make_tuple(kind, elem_bytes, bits));
  if (it != g_tuned.begin()) {
    auto below = std::prev(it);
    if (std::get<0>(below->first) == kind && std::get<1>(below->first) == elem_bytes) return below->second;
  }
  if (it != g_tuned.end() && std::get<0>(it->first) == kind && std::get<1>(it->first) == elem_bytes)
    return it->second;
  return g_cfg;
}
bool g_nontemporal_store = false;
uint32_t g_xcd_mode = 2;  // batched tile ranges per XCD: 0 off, 1 on, 2 automatic
bool g_batch_small = true;  // batched: segments of <= 2^kSmallSegmentBits indices to one wavefront each
// (elem_bytes, domain bits) -> bs_shuffle prefers the staged form (tuned table)
std::map<std::pair<uint32_t, uint32_t>, bool> g_staged;
uint32_t g_staged_policy = 2;  // 0 never, 1 whenever the workspace holds the scratch, 2 as tuned
// look-back watchdog of later launches (spin limit, stall test hook); atomics
// so the entry points can read them without the lock
std::atomic<uint32_t> g_spin_limit{bsd::kSpinLimit};
std::atomic<uint32_t> g_stall_first{0};

bsd::Watchdog current_watchdog() {
  return {g_spin_limit.load(std::memory_order_relaxed), g_stall_first.load(std::memory_order_relaxed)};
}

struct CacheEntry {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::map<std::pair<int, hipStream_t>, CacheEntry> g_cache;
std::map<int, uint32_t> g_num_cus;

uint32_t ceil_log2(uint64_t n) {
  uint32_t k = 0;
  while (k < 64 && (uint64_t(1) << k) < n) ++k;
  return k;
}

uint64_t splitmix64_step(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool valid_elem_bytes(uint32_t eb) { return eb == 1 || eb == 2 || eb == 4 || eb == 8 || eb == 16; }

uint64_t single_capacity(uint64_t n) {
  const uint32_t k = std::max<uint32_t>(ceil_log2(n), BS_MIN_DOMAIN_BITS);
  return ((uint64_t(1) << k) + kMinTile - 1) / kMinTile;
}

// Upper bound on the total tiles of a batch: every non-empty segment pads to
// at most max(16, 2n_s - 1) indices, and rounds its tile count up by one.
uint64_t batch_capacity(uint64_t items, uint32_t segments) {
  return (2 * items + 16ull * segments) / kMinTile + segments + 1;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct BatchLayout {
  size_t status, segs, keys, tile_segment, block_sums, block_bad, total;
  uint64_t capacity;
};

BatchLayout batch_layout(uint64_t items, uint32_t segments) {
  BatchLayout l;
  l.capacity = batch_capacity(items, segments);
  l.status = kHeaderBytes;
  l.segs = align256(l.status + l.capacity * 8);
  l.keys = align256(l.segs + size_t(segments) * sizeof(bsd::SegmentInfo));
  l.tile_segment = align256(l.keys + size_t(segments) * (BS_MAX_ROUNDS + 1) * 4);
  const size_t blocks = (size_t(segments) + bsd::kSegmentsPerBlock - 1) / bsd::kSegmentsPerBlock;
  l.block_sums = align256(l.tile_segment + l.capacity * 4);
  l.block_bad = align256(l.block_sums + blocks * 4);
  l.total = align256(l.block_bad + blocks * 4);
  return l;
}

bs_status device_cus(int dev, uint32_t* cus) {
  auto it = g_num_cus.find(dev);
  if (it != g_num_cus.end()) {
    *cus = it->second;
    return BS_OK;
  }
  int v = 0;
  hipError_t e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e);
  g_num_cus[dev] = uint32_t(v);
  *cus = uint32_t(v);
  return BS_OK;
}

// Resolves the workspace for a call: the caller's, or the library's cache
// entry for (device, stream), grown when too small (never while capturing).
bs_status resolve_workspace(void* user, size_t user_bytes, size_t need, hipStream_t stream, void** ws) {
  if (user) {
    if (user_bytes < need) return BS_ENOMEM;
    if (reinterpret_cast<uintptr_t>(user) % 256 != 0) return BS_EINVAL;
    *ws = user;
    return BS_OK;
  }
  // A captured call must bring its own workspace: the cache may be regrown
  // (freed and reallocated) by a later call, under the captured graph.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(stream, &cap);
  if (e != hipSuccess) return hip_fail(e);
  if (cap != hipStreamCaptureStatusNone) return BS_EINVAL;
  int dev = 0;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  CacheEntry& c = g_cache[{dev, stream}];
  if (c.bytes >= need) {
    *ws = c.ptr;
    return BS_OK;
  }
  size_t bytes = std::max(need, size_t(1) << 20);
  if (c.ptr) {
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipFree(c.ptr);
    c.ptr = nullptr;
    c.bytes = 0;
    if (e != hipSuccess) return hip_fail(e);
  }
  void* p = nullptr;
  e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? BS_ENOMEM : hip_fail(e);
  e = bsd::launch_workspace_init(p, bytes, stream);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e);
  }
  c.ptr = p;
  c.bytes = bytes;
  *ws = p;
  return BS_OK;
}

// Cipher parameters and masked round keys of one call (Sec. 3.2 split, keys
// from SplitMix64 masked to the half width, then a 0).
void setup_cipher(bsd::SingleArgs& a, uint64_t n, uint64_t seed, uint32_t rounds) {
  const uint32_t k = std::max<uint32_t>(ceil_log2(n), BS_MIN_DOMAIN_BITS);
  a.n = n;
  a.domain = uint64_t(1) << k;
  a.cs.w = k / 2;
  a.cs.r = k - a.cs.w;
  a.cs.wmask = (1u << a.cs.w) - 1u;
  a.cs.rmask = uint32_t((uint64_t(1) << a.cs.r) - 1u);
  a.rounds = rounds;
  uint64_t st = seed;
  for (uint32_t r = 0; r < rounds; ++r) a.key[r] = uint32_t(splitmix64_step(st)) & a.cs.wmask;
  a.key[rounds] = 0;
  a.wd = current_watchdog();
}

bool ranges_overlap(const void* a, const void* b, uint64_t bytes) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + bytes && y < x + bytes;
}

// Argument checks shared by the single-shuffle entry points (synchronous,
// before anything is enqueued).
bs_status check_single_args(const void* in, const void* out, uint64_t n, uint32_t elem_bytes, uint32_t rounds) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (ranges_overlap(in, out, n * elem_bytes)) return BS_EALIAS;
  return BS_OK;
}

struct StagedLayout {
  bool ok = false;
  uint32_t k = 0, s = 0, b1 = 0, b2 = 0;
  size_t cnt_a = 0, cnt_b = 0, base_b = 0, idx_a = 0, val_a = 0, idx_b = 0, val_b = 0, total = 0;
};

// Scratch of the staged form: counts, the window prefix, then the two bucket
// arrays (index and record arrays each; the first pass's arrays only when
// there are two distribution passes), every part 256-byte aligned.
StagedLayout staged_layout(uint64_t n, uint32_t elem_bytes) {
  StagedLayout l;
  if (!valid_elem_bytes(elem_bytes) || n == 0 || n > BS_MAX_ITEMS) return l;
  l.k = std::max<uint32_t>(ceil_log2(n), BS_MIN_DOMAIN_BITS);
  if (!bsd::staged_digits(l.k, elem_bytes, &l.s, &l.b1, &l.b2)) return l;
  const uint64_t domain = uint64_t(1) << l.k;
  const uint64_t windows = uint64_t(1) << (l.b1 + l.b2);
  l.cnt_a = 0;
  l.cnt_b = l.cnt_a + align256((uint64_t(1) << l.b1) * 4);
  l.base_b = l.cnt_b + align256(windows * 4);
  l.idx_a = l.base_b + align256(windows * 4);
  // domain * 4 is a multiple of 256 here (k >= 14 whenever b2 > 0), so the
  // value part follows the index part with no gap: 4-byte records keep their
  // first-pass entries as (index, record) pairs over both parts
  l.val_a = l.idx_a + (l.b2 ? align256(domain * 4) : 0);
  l.idx_b = l.val_a + (l.b2 ? align256(domain * elem_bytes) : 0);
  l.val_b = l.idx_b + align256(domain * 2);
  l.total = l.val_b + align256(domain * elem_bytes);
  l.ok = true;
  return l;
}

// The staged form's kernel arguments over a scratch of l.total bytes.
bsd::StagedArgs staged_args(const void* in, void* out, uint64_t n, uint64_t seed, uint32_t rounds, uint8_t* scratch,
                            const StagedLayout& l) {
  bsd::SingleArgs c = {};
  setup_cipher(c, n, seed, rounds);
  bsd::StagedArgs a = {};
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  a.n = n;
  a.cs = c.cs;
  a.k = l.k;
  a.rounds = rounds;
  a.s = l.s;
  a.b1 = l.b1;
  a.b2 = l.b2;
  a.cnt_a = reinterpret_cast<uint32_t*>(scratch + l.cnt_a);
  a.cnt_b = reinterpret_cast<uint32_t*>(scratch + l.cnt_b);
  a.base_b = reinterpret_cast<uint32_t*>(scratch + l.base_b);
  a.idx_a = reinterpret_cast<uint32_t*>(scratch + l.idx_a);
  a.val_a = scratch + l.val_a;
  a.idx_b = reinterpret_cast<uint16_t*>(scratch + l.idx_b);
  a.val_b = scratch + l.val_b;
  std::copy(std::begin(c.key), std::end(c.key), std::begin(a.key));
  return a;
}

// The staged form's launch (arguments checked, scratch of l.total bytes).
bs_status launch_staged_form(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                             uint32_t rounds, uint8_t* scratch, const StagedLayout& l, uint32_t cus, hipStream_t s) {
  const bsd::StagedArgs a = staged_args(in, out, n, seed, rounds, scratch, l);
  const hipError_t e = bsd::launch_staged(a, elem_bytes, cus, s);
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

// Whether bs_shuffle takes the staged form for (elem_bytes, k): policy 1
// always (when the workspace holds its scratch), 2 as the tuned table says
// for the nearest listed class at or below k of that element size, as
// pick_config takes shapes (never while a shape is forced with
// bs_set_config); g_mu held.
bool staged_preferred(uint32_t elem_bytes, uint32_t k) {
  if (g_staged_policy == 1) return true;
  if (g_staged_policy == 0 || g_forced) return false;
  auto it = g_staged.upper_bound({elem_bytes, k});
  if (it == g_staged.begin()) return false;
  --it;
  return it->first.first == elem_bytes && it->second;
}

// One bs_shuffle launch (n > 0, arguments checked); g_mu held.  The fused
// kernel, or the staged form when preferred and the caller's workspace holds
// its scratch after the fused part.
bs_status launch_shuffle(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t rounds,
                         void* workspace, size_t workspace_bytes, hipStream_t s) {
  const uint32_t k = std::max<uint32_t>(ceil_log2(n), BS_MIN_DOMAIN_BITS);
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  const bsd::LaunchConfig cfg = pick_config(0, elem_bytes, k);
  const bool wide = k > 32;
  const uint64_t tile = wide ? 64ull * bsd::kWideWaves * bsd::kWideItems : 64ull * cfg.waves * cfg.items;
  a.num_tiles = uint32_t((a.domain + tile - 1) / tile);
  const size_t need = align256(kHeaderBytes + single_capacity(n) * 8);
  if (workspace && k <= 32 && staged_preferred(elem_bytes, k)) {
    const StagedLayout l = staged_layout(n, elem_bytes);
    if (l.ok && workspace_bytes >= need + l.total) {
      if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return BS_EINVAL;
      int dev = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e != hipSuccess) return hip_fail(e);
      uint32_t cus = 0;
      const bs_status cst = device_cus(dev, &cus);
      if (cst != BS_OK) return cst;
      return launch_staged_form(in, out, n, elem_bytes, seed, rounds, static_cast<uint8_t*>(workspace) + need, l,
                                cus, s);
    }
  }
  void* ws = nullptr;
  bs_status st = resolve_workspace(workspace, workspace_bytes, need, s, &ws);
  if (st != BS_OK) return st;
  a.hdr = static_cast<bsd::WorkspaceHeader*>(ws);
  a.status = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(ws) + kHeaderBytes);
  a.capacity = uint32_t(single_capacity(n));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t cus = 0;
  st = device_cus(dev, &cus);
  if (st != BS_OK) return st;
  e = bsd::launch_single(a, elem_bytes, g_nontemporal_store, cfg, cus, s);
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

// The workspace of bs_shuffle_noalloc is `scratch` (defined above the
// namespace): the header plus one status word per 2,048 padded indices of a
// domain of up to 2^30.  Host code must never pass `scratch` itself to a
// kernel or a copy (in host code the name is a host-side stand-in): it uses
// the device address that hipGetSymbolAddress returns, kept per device.
constexpr size_t kStaticScratchBytes = kHeaderBytes + (size_t(1) << (kStaticMaxDomainBits - 11)) * 8;
static_assert(kStaticScratchBytes == BS_NOALLOC_SCRATCH_BYTES, "scratch size of the ABI");
std::map<int, void*> g_scratch;  // device -> address of `scratch` on that device

// The current device's scratch address (g_mu held).  The first call on a
// device looks the address up and zero-fills the array on `s` (a zero-filled
// workspace is a valid one); that first call must not be captured into a
// graph, because the fill would then only run when the graph does.
bs_status static_scratch(hipStream_t s, void** ws) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) {
    *ws = it->second;
    return BS_OK;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return hip_fail(e);
  if (cap != hipStreamCaptureStatusNone) return BS_EINVAL;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e);
  if (reinterpret_cast<uintptr_t>(p) % 256 != 0) return BS_EINVAL;
  e = bsd::launch_workspace_init(p, kStaticScratchBytes, s);
  if (e != hipSuccess) return hip_fail(e);
  g_scratch[dev] = p;
  *ws = p;
  return BS_OK;
}

}  // namespace

namespace bsd {

ConfigState config_state() {
  std::lock_guard<std::mutex> lock(g_mu);
  return {g_forced, g_cfg};
}

void restore_config_state(const ConfigState& st) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_forced = st.forced;
  g_cfg = st.forced ? st.cfg : g_default_cfg;
}

void set_staged_preference(uint32_t elem_bytes, uint32_t size_bits, bool prefer) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_staged[{elem_bytes, size_bits}] = prefer;
}

std::vector<StagedEntry> staged_snapshot() {
  std::lock_guard<std::mutex> lock(g_mu);
  std::vector<StagedEntry> v;
  for (const auto& kv : g_staged) v.push_back({kv.first.first, kv.first.second, kv.second});
  return v;
}

std::vector<TunedEntry> tuned_snapshot() {
  std::lock_guard<std::mutex> lock(g_mu);
  std::vector<TunedEntry> v;
  for (const auto& kv : g_tuned)
    v.push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second});
  return v;
}

}  // namespace bsd

extern "C" {

const char* bs_status_string(bs_status s) {
  switch (s) {
    case BS_OK: return "BS_OK: success";
    case BS_EINVAL: return "BS_EINVAL: invalid argument";
    case BS_EALIAS: return "BS_EALIAS: input and output overlap";
    case BS_EELEM: return "BS_EELEM: element size must be 1, 2, 4, 8 or 16 bytes and pointers aligned to it";
    case BS_ENOMEM: return "BS_ENOMEM: workspace too small or allocation failed";
    case BS_EHIP: return "BS_EHIP: HIP runtime error";
    case BS_ETIMEOUT: return "BS_ETIMEOUT: look-back wait exceeded its spin limit";
    case BS_ENODEV: return "BS_ENODEV: no HIP device";
    case BS_EDEVICE: return "BS_EDEVICE: batch rejected on the device (bad offsets or too many tiles)";
    default: return "unknown bs_status";
  }
}

int32_t bs_last_hip_error(void) { return g_last_hip_error; }

uint32_t bs_version(void) { return 100; }

uint32_t bs_domain_bits(uint64_t n) { return std::max<uint32_t>(ceil_log2(n), BS_MIN_DOMAIN_BITS); }

bs_status bs_round_keys(uint64_t seed, uint32_t rounds, uint32_t* keys) {
  if (rounds > BS_MAX_ROUNDS || (rounds && !keys)) return BS_EINVAL;
  uint64_t st = seed;
  for (uint32_t r = 0; r < rounds; ++r) keys[r] = uint32_t(splitmix64_step(st));
  return BS_OK;
}

size_t bs_workspace_bytes(uint64_t items, uint32_t num_segments, uint32_t elem_bytes) {
  (void)elem_bytes;
  if (num_segments == 0) return align256(kHeaderBytes + single_capacity(items) * 8);
  return batch_layout(items, num_segments).total;
}

bs_status bs_workspace_init(void* workspace, size_t workspace_bytes, void* stream) {
  if (!workspace || workspace_bytes < kHeaderBytes) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return BS_EINVAL;
  hipError_t e = bsd::launch_workspace_init(workspace, workspace_bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

bs_status bs_workspace_error(void* workspace, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = workspace;
  if (!ws) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_cache.find({dev, s});
    if (it == g_cache.end() || !it->second.ptr) return BS_OK;
    ws = it->second.ptr;
  }
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t err = 0;
  auto* hdr = static_cast<bsd::WorkspaceHeader*>(ws);
  e = hipMemcpy(&err, &hdr->error, sizeof(err), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  if (err) {
    const uint32_t zero = 0;
    e = hipMemcpy(&hdr->error, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (err & bsd::kErrTimeout) return BS_ETIMEOUT;
  if (err & bsd::kErrBadBatch) return BS_EDEVICE;
  return BS_OK;
}

bs_status bs_workspace_error_async(void* workspace, int32_t* status, void* stream) {
  if (!workspace || !status) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0 || reinterpret_cast<uintptr_t>(status) % 4 != 0)
    return BS_EINVAL;
  hipError_t e = bsd::launch_take_error(workspace, status, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

bs_status bs_set_config(uint32_t waves, uint32_t items, uint32_t depth, uint32_t grid_mult) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (waves == 0 && items == 0 && depth == 0 && grid_mult == 0) {
    g_cfg = g_default_cfg;
    g_forced = false;
    return BS_OK;
  }
  bsd::LaunchConfig c = {waves, items, depth, grid_mult};
  if (!bsd::config_supported(c) || (grid_mult > 64 && grid_mult != bsd::kGridOnePerTile)) return BS_EINVAL;
  g_cfg = c;
  g_forced = true;
  return BS_OK;
}

bs_status bs_set_tuned_config(uint32_t kind, uint32_t elem_bytes, uint32_t size_bits, uint32_t waves,
                              uint32_t items, uint32_t depth, uint32_t grid_mult) {
  if (kind > 1 || !valid_elem_bytes(elem_bytes) || size_bits > 40) return BS_EINVAL;
  bsd::LaunchConfig c = {waves, items, depth, grid_mult};
  if (!bsd::config_supported(c) || (grid_mult > 64 && grid_mult != bsd::kGridOnePerTile)) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  g_tuned[std::make_tuple(kind, elem_bytes, size_bits)] = c;
  return BS_OK;
}

bs_status bs_query_config(uint32_t kind, uint32_t elem_bytes, uint64_t items, uint32_t num_segments,
                          uint32_t* waves, uint32_t* items_per_lane, uint32_t* depth, uint32_t* grid_mult) {
  if (kind > 1 || !valid_elem_bytes(elem_bytes) || !waves || !items_per_lane || !depth || !grid_mult)
    return BS_EINVAL;
  if (kind == 1 && num_segments == 0) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  const uint32_t bits = kind == 0 ? bs_domain_bits(items) : ceil_log2((items + num_segments - 1) / num_segments);
  bsd::LaunchConfig c = pick_config(kind, elem_bytes, bits);
  if (kind == 0 && bits > 32) c = {bsd::kWideWaves, bsd::kWideItems, bsd::kDepthCompactPipe, c.grid_mult};
  if (kind == 0 && bits <= 32 && staged_preferred(elem_bytes, bits) && staged_layout(items, elem_bytes).ok)
    c = {0, 0, BS_DEPTH_STAGED, 0};
  if (kind == 1) c = bsd::batch_config(c);
  *waves = c.waves;
  *items_per_lane = c.items;
  *depth = c.depth;
  *grid_mult = c.grid_mult;
  return BS_OK;
}

bs_status bs_clear_tuned_configs(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_tuned.clear();
  g_staged.clear();
  return BS_OK;
}

bs_status bs_get_config(uint32_t* waves, uint32_t* items, uint32_t* depth, uint32_t* grid_mult) {
  if (!waves || !items || !depth || !grid_mult) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  *waves = g_cfg.waves;
  *items = g_cfg.items;
  *depth = g_cfg.depth;
  *grid_mult = g_cfg.grid_mult;
  return BS_OK;
}

bs_status bs_shuffle(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t rounds,
                     void* workspace, size_t workspace_bytes, void* stream) {
  const bs_status st = check_single_args(in, out, n, elem_bytes, rounds);
  if (st != BS_OK || n == 0) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  return launch_shuffle(in, out, n, elem_bytes, seed, rounds, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

bs_status bs_shuffle_noalloc(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                             uint32_t rounds, void* stream) {
  const bs_status st = check_single_args(in, out, n, elem_bytes, rounds);
  if (st != BS_OK || n == 0) return st;
  if (bs_workspace_bytes(n, 0, elem_bytes) > kStaticScratchBytes) return BS_ENOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  void* ws = nullptr;
  const bs_status sst = static_scratch(s, &ws);
  if (sst != BS_OK) return sst;
  return launch_shuffle(in, out, n, elem_bytes, seed, rounds, ws, kStaticScratchBytes, s);
}


bs_status bs_shuffle_batched(const void* in, void* out, const int64_t* offsets, const uint64_t* seeds,
                             uint32_t num_segments, uint64_t total_items, uint32_t elem_bytes, uint32_t rounds,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || total_items > BS_MAX_ITEMS) return BS_EINVAL;
  if (num_segments == 0 || total_items == 0) return BS_OK;
  if (!in || !out || !offsets || !seeds) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (ranges_overlap(in, out, total_items * elem_bytes)) return BS_EALIAS;

  hipStream_t s = static_cast<hipStream_t>(stream);
  const BatchLayout lay = batch_layout(total_items, num_segments);
  if (lay.capacity > 0xFFFFFFFFull) return BS_EINVAL;

  std::lock_guard<std::mutex> lock(g_mu);
  const bsd::LaunchConfig cfg =
      bsd::batch_config(pick_config(1, elem_bytes, ceil_log2((total_items + num_segments - 1) / num_segments)));
  void* ws = nullptr;
  bs_status st = resolve_workspace(workspace, workspace_bytes, lay.total, s, &ws);
  if (st != BS_OK) return st;
  uint8_t* base = static_cast<uint8_t*>(ws);
  bsd::BatchArgs a = {};
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  a.offsets = offsets;
  a.seeds = seeds;
  a.total_items = total_items;
  a.num_segments = num_segments;
  a.rounds = rounds;
  a.capacity = uint32_t(lay.capacity);
  a.tile = 64u * cfg.waves * cfg.items;
  a.nontemporal = g_nontemporal_store ? 1u : 0u;
  a.wd = current_watchdog();
  a.xcd_mode = g_xcd_mode;
  a.small_bits = g_batch_small ? bsd::kSmallSegmentBits : 0u;
  a.hdr = reinterpret_cast<bsd::WorkspaceHeader*>(base);
  a.status = reinterpret_cast<uint64_t*>(base + lay.status);
  a.segs = reinterpret_cast<bsd::SegmentInfo*>(base + lay.segs);
  a.keys = reinterpret_cast<uint32_t*>(base + lay.keys);
  a.tile_segment = reinterpret_cast<uint32_t*>(base + lay.tile_segment);
  a.block_sums = reinterpret_cast<uint32_t*>(base + lay.block_sums);
  a.block_bad = reinterpret_cast<uint32_t*>(base + lay.block_bad);
  a.tables = base + lay.segs;
  a.tables_bytes = lay.total - lay.segs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t cus = 0;
  st = device_cus(dev, &cus);
  if (st != BS_OK) return st;
  e = bsd::launch_batched(a, elem_bytes, cfg, cus, s);
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------- probe entry points --
extern "C" bs_status bs_probe_set_xcd_mode(uint32_t mode) {
  if (mode > 2) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  g_xcd_mode = mode;
  return BS_OK;
}

extern "C" bs_status bs_probe_set_batch_small(uint32_t enable) {
  if (enable > 1) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  g_batch_small = enable != 0;
  return BS_OK;
}

extern "C" bs_status bs_probe_set_watchdog(uint32_t spin_limit, uint32_t stall_first_tile) {
  if (stall_first_tile > 1) return BS_EINVAL;
  g_spin_limit.store(spin_limit ? spin_limit : bsd::kSpinLimit, std::memory_order_relaxed);
  g_stall_first.store(stall_first_tile, std::memory_order_relaxed);
  return BS_OK;
}

extern "C" bs_status bs_probe_set_store_mode(uint32_t nontemporal) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_nontemporal_store = nontemporal != 0;
  return BS_OK;
}

extern "C" bs_status bs_probe_cipher_scan(uint64_t n, uint64_t seed, uint32_t rounds, void* workspace,
                                          size_t workspace_bytes, void* stream) {
  if (rounds > BS_MAX_ROUNDS || n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t k = bs_domain_bits(n);
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  std::lock_guard<std::mutex> lock(g_mu);
  const bsd::LaunchConfig cfg = g_cfg;
  const uint64_t tile = k > 32 ? 64ull * bsd::kWideWaves * bsd::kWideItems : 64ull * cfg.waves * cfg.items;
  a.num_tiles = uint32_t((a.domain + tile - 1) / tile);
  void* ws = nullptr;
  bs_status st = resolve_workspace(workspace, workspace_bytes, bs_workspace_bytes(n, 0, 4), s, &ws);
  if (st != BS_OK) return st;
  a.hdr = static_cast<bsd::WorkspaceHeader*>(ws);
  a.status = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(ws) + kHeaderBytes);
  a.capacity = uint32_t(single_capacity(n));
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t cus = 0;
  st = device_cus(dev, &cus);
  if (st != BS_OK) return st;
  e = bsd::launch_single(a, 0, false, cfg, cus, s);
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

// ---------------------------------------------------- permutation outputs --
namespace {

// Runs one fixed-shape kernel variant over a single shuffle's domain.
bs_status run_variant(bsd::SingleArgs& a, uint32_t variant, uint32_t eb, void* workspace, size_t workspace_bytes,
                      hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_mu);
  const bool wide = a.domain > (uint64_t(1) << 32);
  const uint64_t tile = wide ? 64ull * bsd::kWideWaves * bsd::kWideItems : bsd::kAltTile;
  a.num_tiles = uint32_t((a.domain + tile - 1) / tile);
  void* ws = nullptr;
  bs_status st = resolve_workspace(workspace, workspace_bytes, bs_workspace_bytes(a.n, 0, eb), s, &ws);
  if (st != BS_OK) return st;
  a.hdr = static_cast<bsd::WorkspaceHeader*>(ws);
  a.status = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(ws) + kHeaderBytes);
  a.capacity = uint32_t(single_capacity(a.n));
  a.nontemporal = g_nontemporal_store ? 1u : 0u;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  uint32_t cus = 0;
  st = device_cus(dev, &cus);
  if (st != BS_OK) return st;
  if (variant == bsd::kVarTwoPass) {
    // counts and exclusive prefixes live in the status array (64-bit values
    // with a zero tag, i.e. "nothing yet" to any later look-back)
    a.tile_counts = a.status;
    a.tile_prefix = a.status + a.num_tiles;
    e = bsd::launch_tile_counts(a, s);
    if (e == hipSuccess) e = bsd::launch_tile_prefix(a.tile_counts, a.status + a.num_tiles, a.num_tiles, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  e = bsd::launch_variant(a, variant, eb, cus, s);
  return e == hipSuccess ? BS_OK : (e == hipErrorInvalidValue ? BS_EINVAL : hip_fail(e));
}

}  // namespace

extern "C" bs_status bs_permutation(void* out_idx, uint64_t n, uint32_t index_bytes, uint64_t seed,
                                    uint32_t rounds, void* workspace, size_t workspace_bytes, void* stream) {
  if (index_bytes != 4 && index_bytes != 8) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!out_idx) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(out_idx) % index_bytes) return BS_EELEM;
  if (index_bytes == 4 && n > (uint64_t(1) << 32)) return BS_EINVAL;
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  a.out = static_cast<uint8_t*>(out_idx);
  return run_variant(a, bsd::kVarIndices, index_bytes, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

extern "C" bs_status bs_unshuffle(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                  uint32_t rounds, void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (ranges_overlap(in, out, n * elem_bytes)) return BS_EALIAS;
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  return run_variant(a, bsd::kVarScatter, elem_bytes, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

extern "C" bs_status bs_probe_shuffle_two_pass(const void* in, void* out, uint64_t n, uint32_t elem_bytes,
                                               uint64_t seed, uint32_t rounds, void* workspace,
                                               size_t workspace_bytes, void* stream) {
  if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > (uint64_t(1) << 32)) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (ranges_overlap(in, out, n * elem_bytes)) return BS_EALIAS;
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  return run_variant(a, bsd::kVarTwoPass, elem_bytes, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

extern "C" size_t bs_probe_unfused_scratch_bytes(uint64_t n) {
  const uint64_t domain = uint64_t(1) << bs_domain_bits(n);
  return align256(domain * 4) + align256(n * 4);
}

extern "C" bs_status bs_probe_shuffle_unfused(const void* in, void* out, uint64_t n, uint32_t elem_bytes,
                                              uint64_t seed, uint32_t rounds, void* scratch, size_t scratch_bytes,
                                              void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > (uint64_t(1) << 32)) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out || !scratch) return BS_EINVAL;
  if (scratch_bytes < bs_probe_unfused_scratch_bytes(n)) return BS_ENOMEM;
  if (reinterpret_cast<uintptr_t>(scratch) % 256) return BS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, rounds);
  uint32_t* table = static_cast<uint32_t*>(scratch);
  uint32_t* sources = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(scratch) + align256(a.domain * 4));
  // pass 1: f over the whole padded domain
  hipError_t e = bsd::launch_cipher_table(a, table, s);
  if (e != hipSuccess) return hip_fail(e);
  // pass 2: stream compaction of the images < n into the source list
  a.table = table;
  a.out = reinterpret_cast<uint8_t*>(sources);
  bs_status st = run_variant(a, bsd::kVarFromTable, 4, workspace, workspace_bytes, s);
  if (st != BS_OK) return st;
  // pass 3: the gather
  return bs_probe_gather(in, n, out, sources, n, elem_bytes, stream);
}

// ------------------------------------------------------------ LCG variant --
extern "C" bs_status bs_lcg_params(uint64_t n, uint64_t seed, uint64_t* a, uint64_t* c) {
  if (!a || !c || n > BS_MAX_ITEMS) return BS_EINVAL;
  const uint64_t mask = (uint64_t(1) << bs_domain_bits(n)) - 1;
  uint64_t st = seed;
  *a = (splitmix64_step(st) | 1u) & mask;
  *c = splitmix64_step(st) & mask;
  return BS_OK;
}

extern "C" bs_status bs_shuffle_lcg(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (ranges_overlap(in, out, n * elem_bytes)) return BS_EALIAS;
  bsd::SingleArgs a = {};
  setup_cipher(a, n, seed, 0);
  bs_lcg_params(n, seed, &a.lcg_a, &a.lcg_c);
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  return run_variant(a, bsd::kVarLcg, elem_bytes, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

extern "C" bs_status bs_bijection(const uint64_t* in, uint64_t* out, uint64_t count, uint32_t domain_bits,
                                  uint64_t seed, uint32_t rounds, uint32_t inverse, void* stream) {
  if (domain_bits < 1 || domain_bits > BS_MAX_BIJECTION_BITS || rounds > BS_MAX_ROUNDS || inverse > 1)
    return BS_EINVAL;
  if (count == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % 8 || reinterpret_cast<uintptr_t>(out) % 8) return BS_EELEM;
  bsd::BijectionArgs a = {};
  a.in = in;
  a.out = out;
  a.count = count;
  a.cs.w = domain_bits / 2;
  a.cs.r = domain_bits - a.cs.w;
  a.cs.wmask = (1u << a.cs.w) - 1u;
  a.cs.rmask = (1u << a.cs.r) - 1u;
  a.rounds = rounds;
  a.inverse = inverse;
  uint64_t st = seed;
  for (uint32_t r = 0; r < rounds; ++r) a.key[r] = uint32_t(splitmix64_step(st)) & a.cs.wmask;
  a.key[rounds] = 0;
  const hipError_t e = bsd::launch_bijection(a, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

// ------------------------------------------------- un-shuffle through f^-1 --
namespace {

struct InverseLayout {
  size_t table, tile_counts, tile_prefix, total;  // byte offsets into scratch
};

InverseLayout inverse_layout(uint64_t n) {
  const uint64_t domain = uint64_t(1) << bs_domain_bits(n);
  const uint64_t groups = (domain + bsd::kRankGroup - 1) / bsd::kRankGroup;
  const uint64_t tiles = (domain + bsd::kRankTile - 1) / bsd::kRankTile;
  InverseLayout l;
  l.table = 0;
  l.tile_counts = align256(groups * 8);
  l.tile_prefix = l.tile_counts + align256(tiles * 8);
  l.total = l.tile_prefix + align256(tiles * 8);
  return l;
}

}  // namespace

extern "C" size_t bs_unshuffle_inverse_scratch_bytes(uint64_t n) {
  return n > BS_MAX_ITEMS ? 0 : inverse_layout(n).total;
}

extern "C" bs_status bs_unshuffle_inverse(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                          uint32_t rounds, void* scratch, size_t scratch_bytes, void* stream) {
  if (!valid_elem_bytes(elem_bytes)) return BS_EELEM;
  if (rounds > BS_MAX_ROUNDS || n > BS_MAX_ITEMS) return BS_EINVAL;
  if (n == 0) return BS_OK;
  if (!in || !out || !scratch) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  if (reinterpret_cast<uintptr_t>(scratch) % 256) return BS_EINVAL;
  if (ranges_overlap(in, out, n * elem_bytes)) return BS_EALIAS;
  const InverseLayout l = inverse_layout(n);
  if (scratch_bytes < l.total) return BS_ENOMEM;
  bsd::SingleArgs c = {};
  setup_cipher(c, n, seed, rounds);
  bsd::InverseArgs a = {};
  a.in = static_cast<const uint8_t*>(in);
  a.out = static_cast<uint8_t*>(out);
  a.n = n;
  a.domain = c.domain;
  a.cs = c.cs;
  a.rounds = rounds;
  a.num_tiles = uint32_t((a.domain + bsd::kRankTile - 1) / bsd::kRankTile);
  uint8_t* base = static_cast<uint8_t*>(scratch);
  a.table = reinterpret_cast<uint64_t*>(base + l.table);
  a.tile_counts = reinterpret_cast<uint64_t*>(base + l.tile_counts);
  a.tile_prefix = reinterpret_cast<uint64_t*>(base + l.tile_prefix);
  std::copy(std::begin(c.key), std::end(c.key), std::begin(a.key));
  const hipError_t e = bsd::launch_unshuffle_inverse(a, elem_bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

extern "C" size_t bs_staged_scratch_bytes(uint64_t n, uint32_t elem_bytes) {
  const StagedLayout l = staged_layout(n, elem_bytes);
  return l.ok ? l.total : 0;
}

extern "C" bs_status bs_shuffle_staged(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                       uint32_t rounds, void* scratch, size_t scratch_bytes, void* stream) {
  const bs_status st = check_single_args(in, out, n, elem_bytes, rounds);
  if (st != BS_OK || n == 0) return st;
  const StagedLayout l = staged_layout(n, elem_bytes);
  if (!l.ok) return BS_EINVAL;
  if (!scratch || reinterpret_cast<uintptr_t>(scratch) % 256) return BS_EINVAL;
  if (scratch_bytes < l.total) return BS_ENOMEM;
  {
    // [scratch, scratch + total) against [in, in + n*eb) and [out, out + n*eb)
    const uintptr_t sc = reinterpret_cast<uintptr_t>(scratch);
    const uintptr_t x = reinterpret_cast<uintptr_t>(in), y = reinterpret_cast<uintptr_t>(out);
    const uint64_t bytes = n * elem_bytes;
    if ((sc < x + bytes && x < sc + l.total) || (sc < y + bytes && y < sc + l.total)) return BS_EALIAS;
  }
  int dev = 0;
  uint32_t cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lock(g_mu);
  const bs_status cst = device_cus(dev, &cus);
  if (cst != BS_OK) return cst;
  return launch_staged_form(in, out, n, elem_bytes, seed, rounds, static_cast<uint8_t*>(scratch), l, cus,
                            static_cast<hipStream_t>(stream));
}

// Scratch of the staged un-shuffle: the staged form's, then the kept images
// (one word per padded index, at least one tile), the tiles' kept counts and
// their first ranks.
struct UnshuffleLayout {
  StagedLayout l;
  size_t keys = 0, cnt = 0, base = 0, total = 0;
  uint32_t tiles = 0;
};

UnshuffleLayout unshuffle_staged_layout(uint64_t n, uint32_t elem_bytes) {
  UnshuffleLayout u;
  u.l = staged_layout(n, elem_bytes);
  if (!u.l.ok) return u;
  const uint64_t domain = uint64_t(1) << u.l.k;
  const uint64_t tile = bsd::unshuffle_key_tile(elem_bytes);
  u.tiles = uint32_t(domain > tile ? domain / tile : 1u);
  u.keys = u.l.total;
  u.cnt = u.keys + align256(std::max(domain, tile) * 4);
  u.base = u.cnt + align256(uint64_t(u.tiles) * 4);
  u.total = u.base + align256(uint64_t(u.tiles) * 4);
  return u;
}

extern "C" size_t bs_unshuffle_staged_scratch_bytes(uint64_t n, uint32_t elem_bytes) {
  if (n == 0) return 0;
  const UnshuffleLayout u = unshuffle_staged_layout(n, elem_bytes);
  return u.l.ok ? u.total : 0;
}

extern "C" bs_status bs_unshuffle_staged(const void* in, void* out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                         uint32_t rounds, void* scratch, size_t scratch_bytes, void* stream) {
  const bs_status st = check_single_args(in, out, n, elem_bytes, rounds);
  if (st != BS_OK || n == 0) return st;
  const UnshuffleLayout u = unshuffle_staged_layout(n, elem_bytes);
  if (!u.l.ok) return BS_EINVAL;
  if (!scratch || reinterpret_cast<uintptr_t>(scratch) % 256) return BS_EINVAL;
  if (scratch_bytes < u.total) return BS_ENOMEM;
  {
    const uintptr_t sc = reinterpret_cast<uintptr_t>(scratch);
    const uintptr_t x = reinterpret_cast<uintptr_t>(in), y = reinterpret_cast<uintptr_t>(out);
    const uint64_t bytes = n * elem_bytes;
    if ((sc < x + bytes && x < sc + u.total) || (sc < y + bytes && y < sc + u.total)) return BS_EALIAS;
  }
  int dev = 0;
  uint32_t cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  std::lock_guard<std::mutex> lock(g_mu);
  const bs_status cst = device_cus(dev, &cus);
  if (cst != BS_OK) return cst;
  uint8_t* sb = static_cast<uint8_t*>(scratch);
  const bsd::StagedArgs a = staged_args(in, out, n, seed, rounds, sb, u.l);
  e = bsd::launch_unshuffle_staged(a, reinterpret_cast<uint32_t*>(sb + u.keys), reinterpret_cast<uint32_t*>(sb + u.cnt),
                                   reinterpret_cast<uint32_t*>(sb + u.base), elem_bytes, cus,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BS_OK : hip_fail(e);
}

extern "C" size_t bs_workspace_bytes_staged(uint64_t n, uint32_t elem_bytes) {
  if (!valid_elem_bytes(elem_bytes) || n > BS_MAX_ITEMS) return 0;
  const size_t need = align256(kHeaderBytes + single_capacity(n) * 8);
  const StagedLayout l = staged_layout(n, elem_bytes);
  return l.ok ? need + l.total : need;
}

extern "C" bs_status bs_probe_set_staged_policy(uint32_t mode) {
  if (mode > 2) return BS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  g_staged_policy = mode;
  return BS_OK;
}
