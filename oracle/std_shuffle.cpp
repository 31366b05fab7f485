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
