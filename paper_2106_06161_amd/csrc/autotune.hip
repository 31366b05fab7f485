// Native autotuner of the launch shapes (bs_autotune) and the text format of
// tuned tables (bs_load_tuned_configs, bs_save_tuned_configs).
//
// For every call kind, element size and size class the tuner times each
// compiled tile shape with each grid choice on library-allocated buffers
// (HIP events on a stream of its own, best of three after a warm-up) and
// keeps the fastest.  Shapes never change results, only speed.
//
// Table format (text, one entry per line, '#' starts a comment):
//   arch <gcnArchName without features>
//   rounds <rounds the table was tuned with>
//   <kind> <elem_bytes> <size_bits> <waves> <items> <depth> <grid_mult> [<ms>]
// kind 0 = bs_shuffle keyed by the domain bits k; kind 1 = bs_shuffle_batched
// keyed by ceil(log2(mean segment size)).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "bshuffle.h"
#include "config_state.h"
#include "kernels.h"

namespace {

constexpr uint32_t kTuneRounds = 24;
constexpr uint32_t kMaxSingleBits = 30;
constexpr uint32_t kMinSingleBits = 12;
constexpr uint32_t kMinBatchBits = 8;
constexpr uint32_t kMaxBatchBits = 20;
constexpr uint32_t kBatchItemsBits = 26;  // records per batched tuning launch: 2^26 (less for small max_size_bits)
constexpr uint64_t kMaxTuneBytes = uint64_t(40) << 30;

struct Entry {
  uint32_t kind, elem_bytes, size_bits;
  bsd::LaunchConfig cfg;
  double ms;
};

// A single-shuffle class where the staged form was timed against the fused one.
struct StagedTiming {
  uint32_t elem_bytes, size_bits;
  bool prefer;
  double ms_staged, ms_fused;
};
constexpr uint32_t kMinStagedBits = 20;

std::vector<bsd::LaunchConfig> candidates() {
  std::vector<bsd::LaunchConfig> shapes;
#define BSD_ADD(W, I, D) shapes.push_back({W, I, D, 0});
  BSD_FOR_EACH_SHAPE(BSD_ADD)
#undef BSD_ADD
#define BSD_ADD(W, I)                                  \
  shapes.push_back({W, I, bsd::kDepthCompact, 0});     \
  shapes.push_back({W, I, bsd::kDepthCompactPipe, 0});
  BSD_FOR_EACH_COMPACT_SHAPE(BSD_ADD)
#undef BSD_ADD
  std::vector<bsd::LaunchConfig> out;
  for (const auto& sh : shapes)
    for (uint32_t g : {0u, 1u, 2u, bsd::kGridOnePerTile}) out.push_back({sh.waves, sh.items, sh.depth, g});
  return out;
}

std::string device_arch(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

uint32_t ceil_log2_u64(uint64_t n) {
  uint32_t k = 0;
  while (k < 64 && (uint64_t(1) << k) < n) ++k;
  return k;
}

// SplitMix64 (published definition), for the seeded segment sizes.
uint64_t splitmix64(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool parse_table(const char* path, std::string* arch, std::vector<Entry>* out,
                 std::vector<StagedTiming>* staged) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ls(line);
    std::string first;
    if (!(ls >> first)) continue;
    if (first == "arch") {
      if (!(ls >> *arch)) return false;
      continue;
    }
    if (first == "rounds") continue;
    if (first == "staged") {
      StagedTiming t = {};
      uint32_t prefer = 0;
      if (!(ls >> t.elem_bytes >> t.size_bits >> prefer) || prefer > 1) return false;
      t.prefer = prefer != 0;
      ls >> t.ms_staged >> t.ms_fused;
      staged->push_back(t);
      continue;
    }
    Entry e = {};
    std::istringstream all(line);
    if (!(all >> e.kind >> e.elem_bytes >> e.size_bits >> e.cfg.waves >> e.cfg.items >> e.cfg.depth >>
          e.cfg.grid_mult))
      return false;
    e.ms = 0;
    all >> e.ms;
    out->push_back(e);
  }
  return true;
}

bool write_table(const char* path, const std::string& arch, const std::vector<Entry>& entries,
                 const std::vector<StagedTiming>& staged) {
  FILE* f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "# libbshuffle tuned launch shapes (bs_autotune)\n");
  std::fprintf(f, "arch %s\nrounds %u\n", arch.c_str(), kTuneRounds);
  std::fprintf(f, "# kind elem_bytes size_bits waves items depth grid_mult ms\n");
  for (const auto& e : entries)
    std::fprintf(f, "%u %u %u %u %u %u %u %.4f\n", e.kind, e.elem_bytes, e.size_bits, e.cfg.waves, e.cfg.items,
                 e.cfg.depth, e.cfg.grid_mult, e.ms);
  if (!staged.empty()) std::fprintf(f, "# staged elem_bytes size_bits prefer ms_staged ms_fused\n");
  for (const auto& t : staged)
    std::fprintf(f, "staged %u %u %u %.4f %.4f\n", t.elem_bytes, t.size_bits, t.prefer ? 1u : 0u, t.ms_staged,
                 t.ms_fused);
  return std::fclose(f) == 0;
}

bs_status install(const std::vector<Entry>& entries, const std::vector<StagedTiming>& staged) {
  for (const auto& e : entries)
    if (e.kind > 1 || e.size_bits > 40 || !bsd::config_supported(e.cfg)) return BS_EINVAL;
  for (const auto& t : staged)
    if (t.size_bits > 40 || !(t.elem_bytes == 1 || t.elem_bytes == 2 || t.elem_bytes == 4 || t.elem_bytes == 8 ||
                              t.elem_bytes == 16))
      return BS_EINVAL;
  bs_clear_tuned_configs();
  for (const auto& e : entries) {
    const bs_status st = bs_set_tuned_config(e.kind, e.elem_bytes, e.size_bits, e.cfg.waves, e.cfg.items,
                                             e.cfg.depth, e.cfg.grid_mult);
    if (st != BS_OK) return st;
  }
  for (const auto& t : staged) bsd::set_staged_preference(t.elem_bytes, t.size_bits, t.prefer);
  return BS_OK;
}

// Times fn() on stream s: one warm-up, then the best of three.
template <typename Fn>
bs_status time_best(Fn fn, hipStream_t s, hipEvent_t e0, hipEvent_t e1, double* ms) {
  bs_status st = fn();
  if (st != BS_OK) return st;
  float best = 1e30f;
  for (int i = 0; i < 3; ++i) {
    if (hipEventRecord(e0, s) != hipSuccess) return BS_EHIP;
    st = fn();
    if (st != BS_OK) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return BS_EHIP;
    float t = 0;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return BS_EHIP;
    best = std::min(best, t);
  }
  *ms = best;
  return BS_OK;
}

struct DeviceBuffers {
  void* in = nullptr;
  void* out = nullptr;
  ~DeviceBuffers() {
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
  }
};

bs_status tune_single(uint32_t eb, uint32_t bits, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Entry* best) {
  const uint64_t hi = uint64_t(1) << bits, lo = (hi >> 1) + 1;
  DeviceBuffers b;
  if (hipMalloc(&b.in, hi * eb) != hipSuccess || hipMalloc(&b.out, hi * eb) != hipSuccess) return BS_ENOMEM;
  if (hipMemsetAsync(b.in, 0x5A, hi * eb, s) != hipSuccess) return BS_EHIP;
  best->ms = -1;
  for (const auto& c : candidates()) {
    if (bs_set_config(c.waves, c.items, c.depth, c.grid_mult) != BS_OK) continue;
    double t_hi = 0, t_lo = 0;
    if (time_best([&] { return bs_shuffle(b.in, b.out, hi, eb, 7, kTuneRounds, nullptr, 0, s); }, s, e0, e1,
                  &t_hi) != BS_OK ||
        time_best([&] { return bs_shuffle(b.in, b.out, lo, eb, 7, kTuneRounds, nullptr, 0, s); }, s, e0, e1,
                  &t_lo) != BS_OK)
      continue;
    if (best->ms < 0 || t_hi + t_lo < best->ms) *best = {0, eb, bits, c, t_hi + t_lo};
  }
  return best->ms < 0 ? BS_EHIP : BS_OK;
}

// The staged form on the same two sizes as tune_single, against the best
// fused time; false (nothing timed) when it does not cover the class or its
// scratch does not fit `budget`.
bool tune_staged(uint32_t eb, uint32_t bits, double fused_ms, uint64_t budget, hipStream_t s, hipEvent_t e0,
                 hipEvent_t e1, StagedTiming* out) {
  const uint64_t hi = uint64_t(1) << bits, lo = (hi >> 1) + 1;
  const size_t scratch_bytes = bs_staged_scratch_bytes(hi, eb);
  if (bits < kMinStagedBits || scratch_bytes == 0 || bs_staged_scratch_bytes(lo, eb) == 0 ||
      scratch_bytes + 2 * hi * eb > budget)
    return false;
  DeviceBuffers b;
  void* scratch = nullptr;
  if (hipMalloc(&b.in, hi * eb) != hipSuccess || hipMalloc(&b.out, hi * eb) != hipSuccess ||
      hipMalloc(&scratch, scratch_bytes) != hipSuccess)
    return false;
  bool ok = hipMemsetAsync(b.in, 0x5A, hi * eb, s) == hipSuccess;
  double t_hi = 0, t_lo = 0;
  ok = ok &&
       time_best([&] { return bs_shuffle_staged(b.in, b.out, hi, eb, 7, kTuneRounds, scratch, scratch_bytes, s); },
                 s, e0, e1, &t_hi) == BS_OK &&
       time_best([&] { return bs_shuffle_staged(b.in, b.out, lo, eb, 7, kTuneRounds, scratch, scratch_bytes, s); },
                 s, e0, e1, &t_lo) == BS_OK;
  (void)hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (!ok) return false;
  *out = {eb, bits, t_hi + t_lo < fused_ms, t_hi + t_lo, fused_ms};
  return true;
}

bs_status tune_batched(uint32_t eb, uint32_t bits, uint64_t batch_items, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                       Entry* best) {
  // segment sizes log-uniform over [mean/4, 4*mean], seeded by the size class
  const uint64_t mean = uint64_t(1) << bits;
  const uint32_t count = uint32_t(std::min<uint64_t>(65536, std::max<uint64_t>(16, batch_items / mean)));
  const double l0 = std::log(double(std::max<uint64_t>(1, mean / 4))), l1 = std::log(double(mean * 4));
  std::vector<int64_t> offsets(count + 1, 0);
  std::vector<uint64_t> seeds(count);
  uint64_t st = bits;
  for (uint32_t i = 0; i < count; ++i) {
    const double u = double(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
    offsets[i + 1] = offsets[i] + int64_t(std::floor(std::exp(l0 + u * (l1 - l0))));
    seeds[i] = i + 1;
  }
  const uint64_t total = uint64_t(offsets[count]);
  DeviceBuffers b;
  void *d_off = nullptr, *d_seed = nullptr;
  if (hipMalloc(&b.in, total * eb) != hipSuccess || hipMalloc(&b.out, total * eb) != hipSuccess)
    return BS_ENOMEM;
  if (hipMalloc(&d_off, offsets.size() * 8) != hipSuccess || hipMalloc(&d_seed, seeds.size() * 8) != hipSuccess) {
    if (d_off) (void)hipFree(d_off);
    return BS_ENOMEM;
  }
  bs_status result = BS_OK;
  if (hipMemcpy(d_off, offsets.data(), offsets.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_seed, seeds.data(), seeds.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemsetAsync(b.in, 0x5A, total * eb, s) != hipSuccess)
    result = BS_EHIP;
  best->ms = -1;
  const uint32_t key_bits = ceil_log2_u64((total + count - 1) / count);
  for (const auto& c : candidates()) {
    if (result != BS_OK) break;
    if (bs_set_config(c.waves, c.items, c.depth, c.grid_mult) != BS_OK) continue;
    double t = 0;
    if (time_best(
            [&] {
              return bs_shuffle_batched(b.in, b.out, static_cast<const int64_t*>(d_off),
                                        static_cast<const uint64_t*>(d_seed), count, total, eb, kTuneRounds, nullptr,
                                        0, s);
            },
            s, e0, e1, &t) != BS_OK)
      continue;
    if (best->ms < 0 || t < best->ms) *best = {1, eb, key_bits, c, t};
  }
  (void)hipFree(d_off);
  (void)hipFree(d_seed);
  if (result == BS_OK && best->ms < 0) result = BS_EHIP;
  return result;
}

void report_staged(const StagedTiming& t, bool verbose) {
  if (verbose)
    std::fprintf(stderr, "bs_autotune: staged elem_bytes %u size_bits %u: %.4f ms against %.4f ms fused -> %s\n",
                 t.elem_bytes, t.size_bits, t.ms_staged, t.ms_fused, t.prefer ? "staged" : "fused");
}

void report(const Entry& e, bool verbose) {
  if (verbose)
    std::fprintf(stderr, "bs_autotune: kind %u elem_bytes %u size_bits %u -> %u %u %u %u (%.4f ms)\n", e.kind,
                 e.elem_bytes, e.size_bits, e.cfg.waves, e.cfg.items, e.cfg.depth, e.cfg.grid_mult, e.ms);
}

bs_status tune_device(uint32_t max_bits, bool verbose, std::vector<Entry>* out, std::vector<StagedTiming>* staged) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return BS_EHIP;
  const uint64_t budget = std::min<uint64_t>(free_b / 2, kMaxTuneBytes);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreate(&s) != hipSuccess) return BS_EHIP;
  bs_status st = BS_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = BS_EHIP;
  for (uint32_t eb : {1u, 2u, 4u, 8u, 16u}) {
    for (uint32_t bits = kMinSingleBits; st == BS_OK && bits <= std::min(max_bits, kMaxSingleBits); ++bits) {
      if ((uint64_t(2) << bits) * eb > budget) break;
      Entry e;
      st = tune_single(eb, bits, s, e0, e1, &e);
      if (st == BS_ENOMEM) {  // larger classes do not fit either: keep what is tuned
        st = BS_OK;
        break;
      }
      if (st == BS_OK) {
        report(e, verbose);
        out->push_back(e);
        StagedTiming t;
        if (tune_staged(eb, bits, e.ms, budget, s, e0, e1, &t)) {
          report_staged(t, verbose);
          staged->push_back(t);
        }
      }
    }
    for (uint32_t bits = kMinBatchBits; st == BS_OK && bits <= std::min(max_bits, kMaxBatchBits); ++bits) {
      Entry e;
      st = tune_batched(eb, bits, uint64_t(1) << std::min(kBatchItemsBits, max_bits + 6), s, e0, e1, &e);
      if (st == BS_ENOMEM) {
        st = BS_OK;
        break;
      }
      if (st == BS_OK) {
        report(e, verbose);
        out->push_back(e);
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return st;
}

}  // namespace

extern "C" bs_status bs_load_tuned_configs(const char* path) {
  if (!path) return BS_EINVAL;
  std::string arch;
  std::vector<Entry> entries;
  std::vector<StagedTiming> staged;
  if (!parse_table(path, &arch, &entries, &staged)) return BS_EINVAL;
  return install(entries, staged);
}

extern "C" bs_status bs_save_tuned_configs(const char* path) {
  if (!path) return BS_EINVAL;
  int dev = 0;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess) arch = device_arch(dev);
  std::vector<Entry> entries;
  for (const auto& t : bsd::tuned_snapshot()) entries.push_back({t.kind, t.elem_bytes, t.size_bits, t.cfg, 0.0});
  std::vector<StagedTiming> staged;
  for (const auto& t : bsd::staged_snapshot()) staged.push_back({t.elem_bytes, t.size_bits, t.prefer, 0.0, 0.0});
  return write_table(path, arch, entries, staged) ? BS_OK : BS_EINVAL;
}

extern "C" bs_status bs_autotune(int device, const char* cache_path, uint32_t max_size_bits, uint32_t flags) {
  if (flags & ~uint32_t(BS_AUTOTUNE_VERBOSE)) return BS_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return BS_ENODEV;
  if (device < 0 || device >= count) return BS_EINVAL;
  const std::string arch = device_arch(device);
  if (cache_path) {
    std::string file_arch;
    std::vector<Entry> cached;
    std::vector<StagedTiming> cached_staged;
    if (parse_table(cache_path, &file_arch, &cached, &cached_staged) && file_arch == arch && !cached.empty())
      return install(cached, cached_staged);
  }
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return BS_EHIP;
  const bsd::ConfigState saved = bsd::config_state();
  std::vector<Entry> entries;
  std::vector<StagedTiming> staged;
  bs_status st = tune_device(max_size_bits ? max_size_bits : kMaxSingleBits, flags & BS_AUTOTUNE_VERBOSE, &entries,
                             &staged);
  bsd::restore_config_state(saved);
  (void)hipSetDevice(prev);
  if (st != BS_OK) return st;
  st = install(entries, staged);
  if (st == BS_OK && cache_path && !write_table(cache_path, arch, entries, staged)) st = BS_EINVAL;
  return st;
}
