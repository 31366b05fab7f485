// Un-shuffle in gather form, through the inverse cipher (Sec. 3.2 inverse).
//
// The shuffle wrote y[rank(i)] = x[f(i)] for every kept padded index i.  So
// for each output position p < n of the un-shuffle, i = f^-1(p) is the kept
// index whose image is p, and x[p] = y[rank(i)].  rank(i) is the number of
// kept indices below i, which a per-index scan would need; here it comes from
// a table built in one pass over the padded domain:
//   rank_table_kernel  every entry covers kRankGroup consecutive indices: a
//                      32-bit mask of kept flags and, in the high word, the
//                      kept count before the entry within its rank tile;
//                      tile_counts[tile] = kept count of the tile
//   tile_prefix_kernel exclusive prefix of tile_counts (shared with the
//                      two-pass variant)
//   gather kernel      p -> i = f^-1(p) -> rank = tile_prefix[i / tile]
//                      + entry.high + popcount(entry.low below bit i % 32)
//                      -> out[p] = in[rank]; stores coalesced, two random reads
//                      (entry, record) per output.
// The scatter form (bs_unshuffle) reads coalesced and writes at random; this
// form moves the randomness to the reads, at the price of the table pass.
#include "shuffle_impl.h"

namespace bsd {
namespace {

constexpr int kGatherThreads = 256;
constexpr int kGatherItems = 8;

template <bool ODD>
__global__ __launch_bounds__(kRankThreads) void rank_table_kernel(const InverseArgs a) {
  __shared__ uint32_t wave_totals[kRankThreads / 64];
  constexpr int kSub = 8;  // cipher evaluations interleaved per lane
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t groups = (a.domain + kRankGroup - 1) / kRankGroup;
  for (uint32_t tile = blockIdx.x; tile < a.num_tiles; tile += gridDim.x) {
    const uint64_t g = uint64_t(tile) * kRankThreads + tid;
    const uint64_t first = g * kRankGroup;
    uint32_t bits = 0;
    if (first < a.domain) {
#pragma unroll 1
      for (int s = 0; s < int(kRankGroup) / kSub; ++s) {
        uint32_t L[kSub], R[kSub];
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const uint64_t x = first + uint64_t(s * kSub + j);
          L[j] = uint32_t(x >> a.cs.r) & (a.cs.wmask & 0xFFFFFFu);
          R[j] = uint32_t(x) & a.cs.rmask;
        }
        vp_encrypt<ODD, kSub>(L, R, a.cs, a.rounds, a.key);
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const uint64_t x = first + uint64_t(s * kSub + j);
          const uint64_t y = (uint64_t(L[j]) << a.cs.r) | (R[j] & a.cs.rmask);
          bits |= uint32_t(x < a.domain && y < a.n) << (s * kSub + j);
        }
      }
    }
    const uint32_t count = __builtin_popcount(bits);
    uint32_t incl = count;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, 64);
      if (lane >= uint32_t(off)) incl += t;
    }
    if (lane == 63) wave_totals[wave] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kRankThreads / 64; ++w) {
      before += w < wave ? wave_totals[w] : 0u;
      total += wave_totals[w];
    }
    if (g < groups) a.table[g] = uint64_t(bits) | (uint64_t(before + incl - count) << 32);
    if (tid == 0) a.tile_counts[tile] = total;
    __syncthreads();
  }
}

template <int EB, bool ODD>
__global__ __launch_bounds__(kGatherThreads) void unshuffle_inverse_kernel(const InverseArgs a) {
  using T = typename Payload<EB>::T;
  constexpr uint64_t kStep = uint64_t(kGatherThreads) * kGatherItems;
  for (uint64_t base = uint64_t(blockIdx.x) * kStep + threadIdx.x; base < a.n; base += uint64_t(gridDim.x) * kStep) {
    uint32_t L[kGatherItems], R[kGatherItems];
#pragma unroll
    for (int j = 0; j < kGatherItems; ++j) {
      uint64_t p = base + uint64_t(j) * kGatherThreads;
      p = p < a.n ? p : a.n - 1;  // idle lanes redo the last position and store nothing
      L[j] = uint32_t(p >> a.cs.r) & a.cs.wmask;
      R[j] = uint32_t(p) & a.cs.rmask;
    }
    vp_decrypt<ODD, kGatherItems>(L, R, a.cs, a.rounds, a.key);
    uint64_t idx[kGatherItems], entry[kGatherItems], prefix[kGatherItems];
#pragma unroll
    for (int j = 0; j < kGatherItems; ++j) {
      idx[j] = (uint64_t(L[j]) << a.cs.r) | R[j];
      entry[j] = a.table[idx[j] / kRankGroup];
      prefix[j] = a.tile_prefix[idx[j] / kRankTile];
    }
    T v[kGatherItems];
#pragma unroll
    for (int j = 0; j < kGatherItems; ++j) {
      const uint32_t below = uint32_t(entry[j]) & ((1u << (idx[j] % kRankGroup)) - 1u);
      uint64_t rank = prefix[j] + (entry[j] >> 32) + uint32_t(__builtin_popcount(below));
      rank = rank < a.n ? rank : a.n - 1;  // never past the input, whatever the table holds
      v[j] = load_record<EB>(a.in, rank);
    }
#pragma unroll
    for (int j = 0; j < kGatherItems; ++j) {
      const uint64_t p = base + uint64_t(j) * kGatherThreads;
      if (p < a.n) store_record<EB, false>(a.out, p, v[j]);
    }
  }
}

template <int EB>
void launch_gather(const InverseArgs& a, bool odd, dim3 grid, hipStream_t stream) {
  if (odd)
    hipLaunchKernelGGL((unshuffle_inverse_kernel<EB, true>), grid, dim3(kGatherThreads), 0, stream, a);
  else
    hipLaunchKernelGGL((unshuffle_inverse_kernel<EB, false>), grid, dim3(kGatherThreads), 0, stream, a);
}

}  // namespace

hipError_t launch_unshuffle_inverse(const InverseArgs& a, uint32_t elem_bytes, hipStream_t stream) {
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  const dim3 table_grid(a.num_tiles < 8192u ? a.num_tiles : 8192u);
  if (odd)
    hipLaunchKernelGGL(rank_table_kernel<true>, table_grid, dim3(kRankThreads), 0, stream, a);
  else
    hipLaunchKernelGGL(rank_table_kernel<false>, table_grid, dim3(kRankThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_tile_prefix(a.tile_counts, a.tile_prefix, a.num_tiles, stream);
  if (e != hipSuccess) return e;
  const uint64_t steps = (a.n + uint64_t(kGatherThreads) * kGatherItems - 1) / (uint64_t(kGatherThreads) * kGatherItems);
  const dim3 grid(uint32_t(steps < 65536 ? steps : 65536));
  switch (elem_bytes) {
    case 1: launch_gather<1>(a, odd, grid, stream); break;
    case 2: launch_gather<2>(a, odd, grid, stream); break;
    case 4: launch_gather<4>(a, odd, grid, stream); break;
    case 8: launch_gather<8>(a, odd, grid, stream); break;
    case 16: launch_gather<16>(a, odd, grid, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bsd
