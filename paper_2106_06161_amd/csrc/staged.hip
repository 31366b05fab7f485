// Staged form of the bijective shuffle: the same output as the fused kernel,
// out[rank(i)] = in[f(i)] for every kept padded index i (Algorithm 1), reached
// by streaming passes instead of random gathers.
//
// Algorithm 1 read from the input side: record y < n goes to output position
// rank(f^-1(y)), where f^-1 is the inverse cipher (Sec. 3.2) and rank(i) is
// the number of kept indices below i.  Every kept index has exactly one
// record, so a window of consecutive padded indices holds its records'
// destinations completely, and rank inside a window is a popcount over the
// window's kept indices.  The passes:
//   distribute (first digit)  read in[] in order (coalesced); i = f^-1(y);
//                             append (i, record) to bucket i >> (k - b1)
//   distribute (second digit) per bucket, append to window i >> s
//                             (skipped when one digit reaches the windows)
//   scan                      exclusive prefix of the window counts
//   place                     one workgroup per window of 2^s padded
//                             indices: records to LDS at i mod 2^s, kept
//                             bits, popcount ranks, then out[] in order
// Each pass reads and writes whole cache lines; the random accesses happen
// in LDS.  A bucket's capacity is the number of padded indices it covers, so
// no bucket can overflow; appends within a bucket come from LDS-sorted runs
// placed by one atomic per (tile, bucket), and their order does not matter
// because the place pass orders records by i.
#include "bshuffle.h"
#include "shuffle_impl.h"

namespace bsd {
namespace {

constexpr uint32_t kDistThreads = 256;
constexpr uint32_t kDistItems = 16;
constexpr uint32_t kDistTile = kDistThreads * kDistItems;  // records per distribution tile
constexpr uint32_t kMaxDigitBits = 9;
constexpr uint32_t kMaxDigits = 1u << kMaxDigitBits;
constexpr uint32_t kPlaceThreads = 1024;
constexpr uint32_t kScanThreads = 1024;

// Exclusive scan over a workgroup of THREADS threads; *total gets the sum.
// Uses waves[THREADS / 64] words of LDS; ends with a barrier.
template <uint32_t THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* waves, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= uint32_t(off)) incl += t;
  }
  if (lane == 63) waves[wave] = incl;
  __syncthreads();
  uint32_t before = 0, sum = 0;
#pragma unroll
  for (uint32_t w = 0; w < THREADS / 64; ++w) {
    const uint32_t c = waves[w];
    before += w < wave ? c : 0u;
    sum += c;
  }
  *total = sum;
  __syncthreads();
  return before + incl - v;
}

template <int EB>
struct DistLds {
  uint32_t hist[kMaxDigits];
  uint32_t start[kMaxDigits];
  uint32_t gbase[kMaxDigits];
  uint32_t waves[kDistThreads / 64];
  uint32_t idx[kDistTile];
  typename Payload<EB>::T val[kDistTile];
};

// Sorts one tile of (i, record) entries by digit (i >> shift) & (digits - 1)
// through LDS and appends each digit's run to bucket `bucket_first + digit`
// (capacity `cap` entries each).  pos[j] holds entry j's position within its
// digit (from the LDS histogram) on entry; entries with valid bit j clear
// are skipped.  Called by the whole workgroup.
template <int EB>
__device__ __forceinline__ void append_runs(DistLds<EB>& lds, const uint32_t (&i)[kDistItems],
                                            const typename Payload<EB>::T (&v)[kDistItems],
                                            const uint32_t (&pos)[kDistItems], uint32_t valid, uint32_t shift,
                                            uint32_t digits, uint64_t bucket_first, uint64_t cap,
                                            uint32_t* __restrict__ idx_out, uint8_t* __restrict__ val_out,
                                            uint32_t* __restrict__ counts) {
  const uint32_t tid = threadIdx.x;
  // digit starts within the tile (two digits per thread: digits <= 512)
  const uint32_t d0 = 2 * tid, d1 = 2 * tid + 1;
  const uint32_t h0 = d0 < digits ? lds.hist[d0] : 0u, h1 = d1 < digits ? lds.hist[d1] : 0u;
  uint32_t count;
  const uint32_t s0 = block_exclusive_scan<kDistThreads>(h0 + h1, lds.waves, &count);
  if (d0 < digits) {
    lds.start[d0] = s0;
    if (h0) lds.gbase[d0] = atomicAdd(&counts[bucket_first + d0], h0);
  }
  if (d1 < digits) {
    lds.start[d1] = s0 + h0;
    if (h1) lds.gbase[d1] = atomicAdd(&counts[bucket_first + d1], h1);
  }
  __syncthreads();
#pragma unroll
  for (uint32_t j = 0; j < kDistItems; ++j) {
    if ((valid >> j) & 1u) {
      const uint32_t d = (i[j] >> shift) & (digits - 1);
      const uint32_t p = lds.start[d] + pos[j];
      lds.idx[p] = i[j];
      lds.val[p] = v[j];
    }
  }
  __syncthreads();
  for (uint32_t p = tid; p < count; p += kDistThreads) {
    const uint32_t ii = lds.idx[p];
    const uint32_t d = (ii >> shift) & (digits - 1);
    const uint64_t g = (bucket_first + d) * cap + lds.gbase[d] + (p - lds.start[d]);
    idx_out[g] = ii;
    store_record<EB, false>(val_out, g, lds.val[p]);
  }
  __syncthreads();
}

// First distribution pass: records in input order, i = f^-1(y), digit =
// i >> (k - b1).  With b2 == 0 the digit is already the window.
template <int EB, bool ODD>
__global__ __launch_bounds__(kDistThreads) void staged_first_kernel(const StagedArgs a) {
  using T = typename Payload<EB>::T;
  __shared__ DistLds<EB> lds;
  const uint32_t tid = threadIdx.x;
  const uint32_t digits = 1u << a.b1;
  const uint32_t shift = a.k - a.b1;
  const uint64_t cap = uint64_t(1) << shift;
  uint32_t* idx_out = a.b2 ? a.idx_a : a.idx_b;
  uint8_t* val_out = a.b2 ? a.val_a : a.val_b;
  uint32_t* counts = a.b2 ? a.cnt_a : a.cnt_b;
  const uint64_t tiles = (a.n + kDistTile - 1) / kDistTile;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    for (uint32_t d = tid; d < digits; d += kDistThreads) lds.hist[d] = 0;
    __syncthreads();
    const uint64_t y0 = tile * kDistTile;
    T v[kDistItems];
    uint32_t L[kDistItems], R[kDistItems], pos[kDistItems];
    uint32_t valid = 0;
#pragma unroll
    for (uint32_t j = 0; j < kDistItems; ++j) {
      const uint64_t y = y0 + j * kDistThreads + tid;
      const bool ok = y < a.n;
      const uint64_t yc = ok ? y : a.n - 1;  // idle lanes re-read the last record and keep nothing
      valid |= ok ? (1u << j) : 0u;
      v[j] = load_record<EB>(a.in, yc);
      L[j] = uint32_t(yc >> a.cs.r) & a.cs.wmask;
      R[j] = uint32_t(yc) & a.cs.rmask;
    }
    vp_decrypt<ODD, kDistItems>(L, R, a.cs, a.rounds, a.key);
#pragma unroll
    for (uint32_t j = 0; j < kDistItems; ++j) {
      L[j] = (L[j] << a.cs.r) | R[j];  // the padded index i whose image is y
      pos[j] = ((valid >> j) & 1u) ? atomicAdd(&lds.hist[L[j] >> shift], 1u) : 0u;
    }
    __syncthreads();
    append_runs<EB>(lds, L, v, pos, valid, shift, digits, 0, cap, idx_out, val_out, counts);
  }
}

// Second distribution pass: bucket d1's entries, digit = (i >> s) & (2^b2 -
// 1), appended to window d1 * 2^b2 + digit.  Work item w covers entries
// [c * tile, (c + 1) * tile) of bucket w / chunks.
template <int EB>
__global__ __launch_bounds__(kDistThreads) void staged_second_kernel(const StagedArgs a) {
  using T = typename Payload<EB>::T;
  __shared__ DistLds<EB> lds;
  const uint32_t tid = threadIdx.x;
  const uint32_t digits = 1u << a.b2;
  const uint64_t cap_a = uint64_t(1) << (a.k - a.b1);
  const uint64_t cap_b = uint64_t(1) << a.s;
  const uint64_t chunks = cap_a / kDistTile;
  const uint64_t work = (uint64_t(1) << a.b1) * chunks;
  for (uint64_t w = blockIdx.x; w < work; w += gridDim.x) {
    const uint64_t d1 = w / chunks;
    const uint64_t first = (w % chunks) * kDistTile;
    const uint32_t cnt = a.cnt_a[d1];
    if (first >= cnt) continue;  // uniform across the workgroup
    for (uint32_t d = tid; d < digits; d += kDistThreads) lds.hist[d] = 0;
    __syncthreads();
    T v[kDistItems];
    uint32_t ii[kDistItems], pos[kDistItems];
    uint32_t valid = 0;
#pragma unroll
    for (uint32_t j = 0; j < kDistItems; ++j) {
      const uint64_t e = first + j * kDistThreads + tid;
      const bool ok = e < cnt;
      const uint64_t g = d1 * cap_a + (ok ? e : first);
      valid |= ok ? (1u << j) : 0u;
      ii[j] = a.idx_a[g];
      v[j] = load_record<EB>(a.val_a, g);
    }
#pragma unroll
    for (uint32_t j = 0; j < kDistItems; ++j)
      pos[j] = ((valid >> j) & 1u) ? atomicAdd(&lds.hist[(ii[j] >> a.s) & (digits - 1)], 1u) : 0u;
    __syncthreads();
    append_runs<EB>(lds, ii, v, pos, valid, a.s, digits, d1 << a.b2, cap_b, a.idx_b, a.val_b, a.cnt_b);
  }
}

// Clears the bucket and window counts before a launch's first pass.
__global__ __launch_bounds__(256) void staged_zero_kernel(const StagedArgs a) {
  const uint32_t windows = 1u << (a.b1 + a.b2);
  for (uint32_t q = blockIdx.x * 256 + threadIdx.x; q < windows; q += gridDim.x * 256) a.cnt_b[q] = 0;
  if (a.b2)
    for (uint32_t d = blockIdx.x * 256 + threadIdx.x; d < (1u << a.b1); d += gridDim.x * 256) a.cnt_a[d] = 0;
}

// Exclusive prefix of the window counts (one workgroup).
__global__ __launch_bounds__(kScanThreads) void staged_scan_kernel(const StagedArgs a) {
  __shared__ uint32_t waves[kScanThreads / 64];
  const uint32_t windows = 1u << (a.b1 + a.b2);
  const uint32_t per = (windows + kScanThreads - 1) / kScanThreads;
  const uint32_t first = threadIdx.x * per;
  uint32_t sum = 0;
  for (uint32_t q = first; q < first + per && q < windows; ++q) sum += a.cnt_b[q];
  uint32_t total;
  uint32_t run = block_exclusive_scan<kScanThreads>(sum, waves, &total);
  for (uint32_t q = first; q < first + per && q < windows; ++q) {
    const uint32_t c = a.cnt_b[q];
    a.base_b[q] = run;
    run += c;
  }
}

// Window bits per record size: the window's records fill 64 KB of LDS.
template <int EB>
constexpr uint32_t kWindowBits = EB == 1 ? 16 : EB == 2 ? 15 : EB == 4 ? 14 : EB == 8 ? 13 : 12;

// One workgroup per window q of 2^s padded indices: its records go to LDS at
// i mod 2^s with a kept bit; each thread owns 2^S / kPlaceThreads consecutive
// slots, counts its kept bits, takes its start from a workgroup scan, and
// moves its records to their ranks; the window is then written in order at
// out[base_b[q]].  (s < S only when the whole domain is one window.)
template <int EB>
__global__ __launch_bounds__(kPlaceThreads) void staged_place_kernel(const StagedArgs a) {
  using T = typename Payload<EB>::T;
  constexpr uint32_t S = kWindowBits<EB>;
  constexpr uint32_t W = 1u << S;
  constexpr uint32_t kPer = W / kPlaceThreads;  // slots per thread: 4 .. 64
  static_assert(kPer >= 4 && kPer <= 64, "slots per thread");
  __shared__ T vals[W];
  __shared__ uint32_t bits[W / 32];
  __shared__ uint32_t waves[kPlaceThreads / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t windows = 1u << (a.b1 + a.b2);
  for (uint32_t q = blockIdx.x; q < windows; q += gridDim.x) {
    const uint32_t cnt = a.cnt_b[q];
    const uint64_t base = a.base_b[q];
    for (uint32_t t = tid; t < W / 32; t += kPlaceThreads) bits[t] = 0;
    __syncthreads();
    const uint64_t first = uint64_t(q) << a.s;
    for (uint32_t e = tid; e < cnt; e += kPlaceThreads) {
      const uint32_t il = a.idx_b[first + e] & (W - 1);
      vals[il] = load_record<EB>(a.val_b, first + e);
      atomicOr(&bits[il >> 5], 1u << (il & 31));
    }
    __syncthreads();
    const uint32_t slot0 = tid * kPer;
    uint64_t mine;
    if constexpr (kPer == 64) {
      mine = uint64_t(bits[slot0 >> 5]) | (uint64_t(bits[(slot0 >> 5) + 1]) << 32);
    } else if constexpr (kPer == 32) {
      mine = bits[slot0 >> 5];
    } else {
      mine = (bits[slot0 >> 5] >> (slot0 & 31)) & ((1u << kPer) - 1u);
    }
    T r[kPer];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) r[j] = vals[slot0 + j];
    uint32_t total;
    const uint32_t start = block_exclusive_scan<kPlaceThreads>(uint32_t(__builtin_popcountll(mine)), waves, &total);
    uint32_t p = start;
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      if ((mine >> j) & 1u) vals[p++] = r[j];
    }
    __syncthreads();
    for (uint32_t t = tid; t < cnt; t += kPlaceThreads) store_record<EB, false>(a.out, base + t, vals[t]);
    __syncthreads();
  }
}

template <int EB>
hipError_t launch_staged_eb(const StagedArgs& a, bool odd, uint32_t num_cus, hipStream_t stream) {
  const uint32_t zero_groups = std::max(1u, std::min(256u, (1u << (a.b1 + a.b2)) / 256u));
  hipLaunchKernelGGL(staged_zero_kernel, dim3(zero_groups), dim3(256), 0, stream, a);
  const uint64_t tiles = (a.n + kDistTile - 1) / kDistTile;
  const dim3 g1(uint32_t(tiles < (1u << 20) ? tiles : (1u << 20)));
  if (odd)
    hipLaunchKernelGGL((staged_first_kernel<EB, true>), g1, dim3(kDistThreads), 0, stream, a);
  else
    hipLaunchKernelGGL((staged_first_kernel<EB, false>), g1, dim3(kDistThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.b2) {
    const uint64_t work = (uint64_t(1) << a.b1) * ((uint64_t(1) << (a.k - a.b1)) / kDistTile);
    const dim3 g2(uint32_t(work < (1u << 20) ? work : (1u << 20)));
    hipLaunchKernelGGL((staged_second_kernel<EB>), g2, dim3(kDistThreads), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(staged_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t windows = 1u << (a.b1 + a.b2);
  hipLaunchKernelGGL((staged_place_kernel<EB>), dim3(windows), dim3(kPlaceThreads), 0, stream, a);
  (void)num_cus;
  return hipGetLastError();
}

}  // namespace

uint32_t staged_window_bits(uint32_t elem_bytes) {
  switch (elem_bytes) {
    case 1: return kWindowBits<1>;
    case 2: return kWindowBits<2>;
    case 4: return kWindowBits<4>;
    case 8: return kWindowBits<8>;
    case 16: return kWindowBits<16>;
    default: return 0;
  }
}

// Splits the k - s digit bits over one or two distribution passes (at most
// kMaxDigitBits each).  False when the domain is outside what the staged
// form covers.
bool staged_digits(uint32_t k, uint32_t elem_bytes, uint32_t* s, uint32_t* b1, uint32_t* b2) {
  const uint32_t ws = staged_window_bits(elem_bytes);
  if (ws == 0 || k > 32) return false;
  const uint32_t win = k < ws ? k : ws;
  const uint32_t nb = k - win;
  if (nb > 2 * kMaxDigitBits) return false;
  *s = win;
  if (nb <= kMaxDigitBits) {
    *b1 = nb;
    *b2 = 0;
  } else {
    *b1 = (nb + 1) / 2;
    *b2 = nb - *b1;
  }
  // the second pass reads first-pass buckets in whole distribution tiles
  if (*b2 && (uint64_t(1) << (k - *b1)) < kDistTile) return false;
  return true;
}

hipError_t launch_staged(const StagedArgs& a, uint32_t elem_bytes, uint32_t num_cus, hipStream_t stream) {
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  switch (elem_bytes) {
    case 1: return launch_staged_eb<1>(a, odd, num_cus, stream);
    case 2: return launch_staged_eb<2>(a, odd, num_cus, stream);
    case 4: return launch_staged_eb<4>(a, odd, num_cus, stream);
    case 8: return launch_staged_eb<8>(a, odd, num_cus, stream);
    case 16: return launch_staged_eb<16>(a, odd, num_cus, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bsd
