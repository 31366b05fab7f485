// CPU timing reference (TEST / BENCHMARK INFRASTRUCTURE ONLY): the C++
// standard library's Fisher-Yates shuffle driven by a 64-bit Mersenne
// twister, single thread.  Used by the benchmark's CPU-baseline leg next to
// the oracle; not part of the method and not part of the product path.
#include <algorithm>
#include <cstdint>
#include <random>

extern "C" void cpu_std_shuffle_u32(uint32_t* data, uint64_t n, uint64_t seed) {
  std::mt19937_64 gen(seed);
  std::shuffle(data, data + n, gen);
}

// count rows of arange(n), row p shuffled with std::mt19937_64(first_seed + p):
// the control sample of the statistical tests (a generator that should pass).
extern "C" void cpu_std_permutations_u32(uint32_t* out, uint64_t n, uint64_t count, uint64_t first_seed) {
  for (uint64_t p = 0; p < count; ++p) {
    uint32_t* row = out + p * n;
    for (uint64_t i = 0; i < n; ++i) row[i] = static_cast<uint32_t>(i);
    std::mt19937_64 gen(first_seed + p);
    std::shuffle(row, row + n, gen);
  }
}
