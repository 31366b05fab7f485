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

constexpr uint32_t kMaxDigitBits = 9;
constexpr uint32_t kMaxDigits = 1u << kMaxDigitBits;
constexpr uint32_t kPlaceThreads = 1024;
constexpr uint32_t kScanThreads = 1024;

// Tile shapes of the distribution passes (PASS 1: first pass, PASS 3: first
// pass with two workgroups per CU, PASS 2: second pass).  The first pass takes
// as many records per tile as its LDS staging area holds with one workgroup
// per CU: every record of a tile that lands in the same bucket shares one
// global reservation, and all tiles reserve from the same 2^b1 counters, so
// large tiles keep those few counters from serializing the pass.  Its other
// shape (PASS 3: 8,192-record tiles on 512 threads) runs two workgroups per
// CU, whose phases overlap the cipher with the other's memory work; it pays
// off once the inverse cipher is long (a round costs five instructions for
// even k, eight for odd k), as long as 2^b1 <= 256 keeps its runs at 32
// records or more; with a short cipher the larger tiles' fewer reservations
// win.  The
// second pass spreads its reservations over 2^(b1 + b2) window counters and
// uses 8,192-record tiles with two workgroups per CU.
template <int EB, int PASS>
struct DistShape {
  static constexpr uint32_t kThreads =
      PASS == 1 ? 1024u : PASS == 3 ? (EB <= 4 ? 512u : 1024u) : (EB <= 8 ? 512u : 1024u);
  static constexpr uint32_t kTile = PASS != 2 ? (PASS == 3 && EB <= 4 ? 8192u : EB <= 4 ? 16384u : EB == 8 ? 8192u : 4096u)
                                              : (EB <= 4 ? 8192u : 4096u);
  static constexpr uint32_t kItems = kTile / kThreads;
  static constexpr uint32_t kDigitsPerThread = (kMaxDigits + kThreads - 1) / kThreads;
  // wavefronts per SIMD the register budget must allow (two workgroups per CU
  // for the PASS 3 shape, one otherwise)
  static constexpr uint32_t kMinWavesPerEU = PASS == 3 && EB <= 4 ? 2u * kThreads / 256u : kThreads / 256u;
};
constexpr uint32_t kMaxFirstTile = 16384;

// Buffer resource word 3 for raw (unformatted, unswizzled) 32-bit-format
// buffer accesses on gfx9-family chips.
constexpr int kBufferWord3 = 0x00020000;

template <int EB>
__device__ __forceinline__ typename Payload<EB>::T buffer_load_record(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                                      uint32_t soff) {
  if constexpr (EB == 1) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
  } else if constexpr (EB == 2) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
  } else if constexpr (EB == 4) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  } else if constexpr (EB == 8) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return uint64_t(w[0]) | (uint64_t(w[1]) << 32);
  } else {
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return Rec16{uint64_t(w[0]) | (uint64_t(w[1]) << 32), uint64_t(w[2]) | (uint64_t(w[3]) << 32)};
  }
}

// The valid-item mask of a whole tile.
template <typename S>
constexpr uint32_t kAllItems = S::kItems >= 32 ? ~0u : (1u << S::kItems) - 1u;

// Two-pass bucket entries of 4-byte records are written as one 8-byte pair
// (padded index, record) at idx_a[2 e] (the index and record arrays are
// adjacent in the scratch): one store per entry in the first pass and one
// load in the second, instead of two each.
template <int EB>
constexpr bool kPairedBuckets = EB == 4;

// Waits for every vector memory operation this wavefront has issued
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).  Loads,
// stores and atomics share one in-order counter, so a load consumed after
// a loop of stores of unknown length makes the compiler wait for all of them:
// waiting here, before the stores are issued, ends the loads' wait while
// nothing else is in flight, and the stores then drain while the next work
// proceeds.
__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Inclusive scan over the 64 lanes of a wavefront with DPP moves (no LDS
// traffic, no lane-address registers): shifts by 1, 2, 4 and 8 within each
// row of 16 lanes, then lane 15 of each row added into the next row and lane
// 31 into the upper half.  Lanes whose DPP source is outside the row, and
// rows the row mask leaves out, receive the 0 given as the old value.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x111, 0xf, 0xf, false));  // row_shr:1
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x112, 0xf, 0xf, false));  // row_shr:2
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x114, 0xf, 0xf, false));  // row_shr:4
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x118, 0xf, 0xf, false));  // row_shr:8
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x142, 0xa, 0xf, false));  // row_bcast:15, rows 1, 3
  v += uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x143, 0xc, 0xf, false));  // row_bcast:31, rows 2, 3
  return v;
}

// Exclusive scan over a workgroup of THREADS threads; *total gets the sum.
// Uses waves[THREADS / 64] words of LDS; ends with a barrier.
template <uint32_t THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* waves, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_inclusive_scan(v);
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

template <int EB, typename S>
struct DistLds {
  uint32_t hist[kMaxDigits];
  uint32_t start[kMaxDigits];
  uint32_t gbase[kMaxDigits];
  uint32_t waves[S::kThreads / 64];
  // the tile's entries in digit order: (index, record) pairs for 4-byte
  // records (one 8-byte LDS access each), separate arrays otherwise
  static constexpr bool kPaired = EB == 4;
  u32x2 pair[kPaired ? S::kTile : 1];
  uint32_t idx[kPaired ? 1 : S::kTile];
  typename Payload<EB>::T val[kPaired ? 1 : S::kTile];
};

// One distribution tile of (i, record) entries, sorted by digit
// (i >> shift) & (digits - 1) through LDS and appended to bucket
// `bucket_first + digit` (capacity `cap` entries each), in four steps so a
// caller can overlap the global reservations' latency with other work:
//   reserve_runs    scan of the LDS histogram -> digit starts in the tile;
//                   one global atomic per digit reserves its run (results
//                   stay in registers)
//   stage_entries   entries to LDS at start[digit] + their position
//   publish_bases   the reserved run bases to LDS (waits for the atomics)
//   write_runs      each run to its bucket; consecutive threads write
//                   consecutive entries of a run.  Windows (the second
//                   level, or the first with one pass) keep only the low 16
//                   bits of i: the place pass needs i mod 2^s, s <= 16.
template <typename S>
struct Reservation {
  uint32_t h[S::kDigitsPerThread];  // this thread's digits: entries in the tile,
  uint32_t s[S::kDigitsPerThread];  // their first position in the tile
  uint32_t g[S::kDigitsPerThread];  // and the reserved position in their bucket
  uint32_t count;                   // entries in the tile
};

template <int EB, typename S>
__device__ __forceinline__ void reserve_runs(DistLds<EB, S>& lds, Reservation<S>& r, uint32_t digits,
                                             uint64_t bucket_first, uint32_t* __restrict__ counts) {
  constexpr uint32_t kPer = S::kDigitsPerThread;
  const uint32_t tid = threadIdx.x;
  uint32_t sum = 0;
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t d = tid * kPer + j;
    r.h[j] = d < digits ? lds.hist[d] : 0u;
    sum += r.h[j];
  }
  uint32_t run = block_exclusive_scan<S::kThreads>(sum, lds.waves, &r.count);
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t d = tid * kPer + j;
    r.s[j] = run;
    if (d < digits) {
      lds.start[d] = run;
      r.g[j] = r.h[j] ? atomicAdd(&counts[bucket_first + d], r.h[j]) : 0u;
    }
    run += r.h[j];
  }
  __syncthreads();
}

template <int EB, typename S>
__device__ __forceinline__ void stage_entries(DistLds<EB, S>& lds, const uint32_t (&i)[S::kItems],
                                              const typename Payload<EB>::T (&v)[S::kItems],
                                              const uint32_t (&pos)[S::kItems], uint32_t valid, uint32_t shift,
                                              uint32_t digits) {
  const uint32_t dbits = __builtin_ctz(digits);
  auto put = [&](uint32_t j) {
    const uint32_t p = lds.start[__builtin_amdgcn_ubfe(i[j], shift, dbits)] + pos[j];
    if constexpr (DistLds<EB, S>::kPaired) {
      lds.pair[p] = u32x2{i[j], v[j]};
    } else {
      lds.idx[p] = i[j];
      lds.val[p] = v[j];
    }
  };
  if (valid == kAllItems<S>) {  // a whole tile: no per-item checks
#pragma unroll
    for (uint32_t j = 0; j < S::kItems; ++j) put(j);
  } else {
#pragma unroll
    for (uint32_t j = 0; j < S::kItems; ++j)
      if ((valid >> j) & 1u) put(j);
  }
}

// gbase[d] = the bucket-array entry of the tile's position 0 in digit d's
// run: (first bucket + d) * capacity + reserved position - start of the run
// in the tile, mod 2^32 (every bucket-array entry index is below 2^32: the
// domain is at most 2^32), so an entry's destination is gbase[d] + position.
template <int EB, typename S>
__device__ __forceinline__ void publish_bases(DistLds<EB, S>& lds, const Reservation<S>& r, uint32_t digits,
                                              uint32_t bucket_first, uint32_t cap) {
  constexpr uint32_t kPer = S::kDigitsPerThread;
#pragma unroll
  for (uint32_t j = 0; j < kPer; ++j) {
    const uint32_t d = threadIdx.x * kPer + j;
    if (d < digits && r.h[j]) lds.gbase[d] = (bucket_first + d) * cap + r.g[j] - r.s[j];
  }
  __syncthreads();
}

// Each run to its bucket: thread t writes tile positions t, t + T, ... (T
// threads), four at a time: the LDS reads of a group first (positions past
// the count re-read position 0), then the destinations, then the stores under
// the count.  WIN: windows keep only the low 16 bits of i.
template <int EB, typename S, bool WIN>
__device__ __forceinline__ void write_runs(DistLds<EB, S>& lds, uint32_t count, uint32_t shift, uint32_t digits,
                                           void* __restrict__ idx_out, uint8_t* __restrict__ val_out) {
  using T = typename Payload<EB>::T;
  constexpr uint32_t kGroup = S::kItems < 4 ? S::kItems : 4;
  if (count == S::kTile) {
    // a whole tile: no position checks, LDS reads at fixed offsets from the
    // group's first position
    const uint32_t dbits = __builtin_ctz(digits);
#pragma unroll 1
    for (uint32_t j0 = 0; j0 < S::kItems; j0 += kGroup) {
      const uint32_t p0 = j0 * S::kThreads + threadIdx.x;
      uint32_t ii[kGroup], g[kGroup];
      T v[kGroup];
#pragma unroll
      for (uint32_t j = 0; j < kGroup; ++j) {
        if constexpr (DistLds<EB, S>::kPaired) {
          const u32x2 e = lds.pair[p0 + j * S::kThreads];
          ii[j] = e.x;
          v[j] = e.y;
        } else {
          ii[j] = lds.idx[p0 + j * S::kThreads];
          v[j] = lds.val[p0 + j * S::kThreads];
        }
      }
#pragma unroll
      for (uint32_t j = 0; j < kGroup; ++j)
        g[j] = lds.gbase[__builtin_amdgcn_ubfe(ii[j], shift, dbits)] + p0 + j * S::kThreads;
#pragma unroll
      for (uint32_t j = 0; j < kGroup; ++j) {
        if constexpr (WIN) {
          static_cast<uint16_t*>(idx_out)[g[j]] = uint16_t(ii[j]);
          store_record<EB, false>(val_out, g[j], v[j]);
        } else if constexpr (kPairedBuckets<EB>) {
          static_cast<u32x2*>(idx_out)[g[j]] = u32x2{ii[j], v[j]};
        } else {
          static_cast<uint32_t*>(idx_out)[g[j]] = ii[j];
          store_record<EB, false>(val_out, g[j], v[j]);
        }
      }
    }
    __syncthreads();
    return;
  }
#pragma unroll 1
  for (uint32_t j0 = 0; j0 < S::kItems; j0 += kGroup) {
    uint32_t ii[kGroup], g[kGroup];
    T v[kGroup];
#pragma unroll
    for (uint32_t j = 0; j < kGroup; ++j) {
      const uint32_t p = (j0 + j) * S::kThreads + threadIdx.x;
      const uint32_t pc = p < count ? p : 0u;
      if constexpr (DistLds<EB, S>::kPaired) {
        const u32x2 e = lds.pair[pc];
        ii[j] = e.x;
        v[j] = e.y;
      } else {
        ii[j] = lds.idx[pc];
        v[j] = lds.val[pc];
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kGroup; ++j)
      g[j] = lds.gbase[(ii[j] >> shift) & (digits - 1)] + (j0 + j) * S::kThreads + threadIdx.x;
#pragma unroll
    for (uint32_t j = 0; j < kGroup; ++j) {
      if ((j0 + j) * S::kThreads + threadIdx.x < count) {
        if constexpr (WIN) {
          static_cast<uint16_t*>(idx_out)[g[j]] = uint16_t(ii[j]);
          store_record<EB, false>(val_out, g[j], v[j]);
        } else if constexpr (kPairedBuckets<EB>) {
          static_cast<u32x2*>(idx_out)[g[j]] = u32x2{ii[j], v[j]};
        } else {
          static_cast<uint32_t*>(idx_out)[g[j]] = ii[j];
          store_record<EB, false>(val_out, g[j], v[j]);
        }
      }
    }
  }
  __syncthreads();
}

// First distribution pass: records in input order, i = f^-1(y), digit =
// i >> (k - b1).  With b2 == 0 the digit is already the window.  Persistent:
// a workgroup walks tiles gridDim.x apart; the next tile's loads and cipher
// (the pass's VALU work) run while the current tile's reservations are in
// flight, and the loads stay in flight through the current tile's writes.
template <int EB, typename S>
__device__ __forceinline__ uint32_t load_tile(typename Payload<EB>::T (&v)[S::kItems], uint32_t (&L)[S::kItems],
                                              uint32_t (&R)[S::kItems], const StagedArgs& a, uint64_t tile) {
  // 32-bit lane arithmetic: the staged form's domain is at most 2^32, so
  // every y fits; the tile's first record and its remaining count are uniform
  const uint64_t y0 = tile * S::kTile;
  const uint64_t left64 = a.n - y0;
  const uint32_t left = left64 < S::kTile ? uint32_t(left64) : S::kTile;  // >= 1
  const uint8_t* base = a.in + y0 * EB;
  if (left == S::kTile) {
    // a whole tile: buffer loads over the tile's bytes, the same lane offset
    // for every item and the item's offset in a scalar register (every
    // access inside the tile)
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), 0, int(S::kTile * EB), kBufferWord3);
#pragma unroll
    for (uint32_t j = 0; j < S::kItems; ++j) {
      v[j] = buffer_load_record<EB>(rsrc, threadIdx.x * EB, j * S::kThreads * EB);
      const uint32_t y = uint32_t(y0) + j * S::kThreads + threadIdx.x;
      L[j] = __builtin_amdgcn_ubfe(y, a.cs.r, a.cs.w);
      R[j] = y & a.cs.rmask;
    }
    return kAllItems<S>;
  }
  uint32_t valid = 0;
#pragma unroll
  for (uint32_t j = 0; j < S::kItems; ++j) {
    const uint32_t off = j * S::kThreads + threadIdx.x;
    const bool ok = off < left;
    const uint32_t oc = ok ? off : left - 1;  // idle lanes re-read the tile's last record and keep nothing
    valid |= ok ? (1u << j) : 0u;
    v[j] = load_record<EB>(base + oc * uint32_t(EB), 0);  // uniform base + 32-bit lane offset
    const uint32_t y = uint32_t(y0) + oc;
    L[j] = __builtin_amdgcn_ubfe(y, a.cs.r, a.cs.w);
    R[j] = y & a.cs.rmask;
  }
  return valid;
}

template <int EB, bool ODD, bool SMALL>
__global__ __launch_bounds__((DistShape<EB, SMALL ? 3 : 1>::kThreads), (DistShape<EB, SMALL ? 3 : 1>::kMinWavesPerEU))
void staged_first_kernel(const StagedArgs a) {
  using S = DistShape<EB, SMALL ? 3 : 1>;
  using T = typename Payload<EB>::T;
  constexpr uint32_t kItems = S::kItems;
  __shared__ DistLds<EB, S> lds;
  const uint32_t tid = threadIdx.x;
  const uint32_t digits = 1u << a.b1;
  const uint32_t shift = a.k - a.b1;
  const uint64_t cap = uint64_t(1) << shift;
  const bool windows = a.b2 == 0;
  void* idx_out = windows ? static_cast<void*>(a.idx_b) : static_cast<void*>(a.idx_a);
  uint8_t* val_out = windows ? a.val_b : a.val_a;
  uint32_t* counts = windows ? a.cnt_b : a.cnt_a;
  const uint64_t tiles = (a.n + S::kTile - 1) / S::kTile;
  uint64_t tile = blockIdx.x;
  if (tile >= tiles) return;
  T v[kItems];
  uint32_t L[kItems], R[kItems], pos[kItems];
  uint32_t valid = load_tile<EB, S>(v, L, R, a, tile);
  // the cipher runs at a raised wave priority: the SIMDs then issue its VALU
  // work ahead of the other workgroup's histogram, staging and run writes,
  // whose few instructions mostly wait on LDS and memory latency anyway
  __builtin_amdgcn_s_setprio(2);
  vp_decrypt<ODD, kItems>(L, R, a.cs, a.rounds, a.key);
  __builtin_amdgcn_s_setprio(0);
  // loads complete on both paths into the loop (see the wait before the
  // stores), so staging never waits on the previous tile's stores
  wait_vector_memory();
  for (;;) {
    for (uint32_t d = tid; d < digits; d += S::kThreads) lds.hist[d] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) L[j] = (L[j] << a.cs.r) | R[j];  // the padded index i whose image is y
    if (valid == kAllItems<S>) {
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j) pos[j] = atomicAdd(&lds.hist[L[j] >> shift], 1u);
    } else {
#pragma unroll
      for (uint32_t j = 0; j < kItems; ++j)
        pos[j] = ((valid >> j) & 1u) ? atomicAdd(&lds.hist[L[j] >> shift], 1u) : 0u;
    }
    __syncthreads();
    Reservation<S> res;
    reserve_runs<EB, S>(lds, res, digits, 0, counts);
    stage_entries<EB, S>(lds, L, v, pos, valid, shift, digits);
    const uint64_t next = tile + gridDim.x;
    const bool more = next < tiles;
    if (more) {
      valid = load_tile<EB, S>(v, L, R, a, next);
      __builtin_amdgcn_s_setprio(2);
      vp_decrypt<ODD, kItems>(L, R, a.cs, a.rounds, a.key);
      __builtin_amdgcn_s_setprio(0);
    }
    publish_bases<EB, S>(lds, res, digits, 0u, uint32_t(cap));
    // the next tile's loads (issued before its cipher) are in; the stores
    // below then do not hold up the next tile's staging
    wait_vector_memory();
    if (windows)
      write_runs<EB, S, true>(lds, res.count, shift, digits, idx_out, val_out);
    else
      write_runs<EB, S, false>(lds, res.count, shift, digits, idx_out, val_out);
    if (!more) break;
    tile = next;
  }
}

// Second distribution pass: bucket d1's entries, digit = (i >> s) & (2^b2 -
// 1), appended to window d1 * 2^b2 + digit.  Workgroup w covers entries
// [c * tile, (c + 1) * tile) of bucket w / chunks, c = w mod chunks;
// workgroups past a bucket's count exit at once (about half of them: a
// bucket holds the kept share of its capacity).  Consecutive workgroups
// share a bucket, so the workgroups in flight append to the same windows and
// their runs fill whole lines in L2 before they are written back.
template <int EB>
__global__ __launch_bounds__((DistShape<EB, 2>::kThreads)) void staged_second_kernel(const StagedArgs a) {
  using S = DistShape<EB, 2>;
  using T = typename Payload<EB>::T;
  constexpr uint32_t kItems = S::kItems;
  __shared__ DistLds<EB, S> lds;
  const uint32_t tid = threadIdx.x;
  const uint32_t digits = 1u << a.b2;
  const uint64_t cap_a = uint64_t(1) << (a.k - a.b1);
  const uint64_t cap_b = uint64_t(1) << a.s;
  const uint64_t chunks = cap_a / S::kTile;
  const uint64_t d1 = blockIdx.x / chunks;
  const uint64_t first = (blockIdx.x % chunks) * S::kTile;
  const uint32_t cnt = a.cnt_a[d1];
  if (first >= cnt) return;  // uniform across the workgroup
  for (uint32_t d = tid; d < digits; d += S::kThreads) lds.hist[d] = 0;
  T v[kItems];
  uint32_t ii[kItems], pos[kItems];
  uint32_t valid = 0;
  // the tile's entries from a uniform base and 32-bit lane offsets
  const uint64_t g0 = d1 * cap_a + first;
  const uint32_t* __restrict__ ti = a.idx_a + g0;
  const uint8_t* tv = a.val_a + g0 * EB;
  const u32x2* __restrict__ tp = reinterpret_cast<const u32x2*>(a.idx_a) + g0;
  const uint32_t left = cnt - uint32_t(first);  // >= 1
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    const uint32_t off = j * S::kThreads + tid;
    const bool ok = off < left;
    valid |= ok ? (1u << j) : 0u;
    const uint32_t oc = ok ? off : 0u;  // idle lanes re-read the tile's first entry
    if constexpr (kPairedBuckets<EB>) {
      const u32x2 r = tp[oc];
      ii[j] = r.x;
      v[j] = r.y;
    } else {
      ii[j] = ti[oc];
      v[j] = load_record<EB>(tv + oc * uint32_t(EB), 0);
    }
  }
  __syncthreads();  // the histogram is cleared
  if (valid == kAllItems<S>) {
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j) pos[j] = atomicAdd(&lds.hist[__builtin_amdgcn_ubfe(ii[j], a.s, a.b2)], 1u);
  } else {
#pragma unroll
    for (uint32_t j = 0; j < kItems; ++j)
      pos[j] = ((valid >> j) & 1u) ? atomicAdd(&lds.hist[__builtin_amdgcn_ubfe(ii[j], a.s, a.b2)], 1u) : 0u;
  }
  __syncthreads();
  Reservation<S> res;
  reserve_runs<EB, S>(lds, res, digits, d1 << a.b2, a.cnt_b);
  stage_entries<EB, S>(lds, ii, v, pos, valid, a.s, digits);
  publish_bases<EB, S>(lds, res, digits, uint32_t(d1 << a.b2), uint32_t(cap_b));
  write_runs<EB, S, true>(lds, res.count, a.s, digits, a.idx_b, a.val_b);
}

// Clears the bucket and window counts before a launch's first pass.
__global__ __launch_bounds__(256) void staged_zero_kernel(const StagedArgs a) {
  const uint32_t windows = 1u << (a.b1 + a.b2);
  for (uint32_t q = blockIdx.x * 256 + threadIdx.x; q < windows; q += gridDim.x * 256) a.cnt_b[q] = 0;
  if (a.b2)
    for (uint32_t d = blockIdx.x * 256 + threadIdx.x; d < (1u << a.b1); d += gridDim.x * 256) a.cnt_a[d] = 0;
}

// Exclusive prefix of the window counts (one workgroup).  Each thread owns
// `per` consecutive windows (a power of two: the window count is one, and
// with fewer windows than threads only the first threads own one); with
// per >= 4 it moves them as 16-byte vectors.  The counts are read through a
// restrict pointer so the second sweep's loads need not wait for the
// first stores of the bases.
__global__ __launch_bounds__(kScanThreads) void staged_scan_kernel(const StagedArgs a) {
  __shared__ uint32_t waves[kScanThreads / 64];
  const uint32_t windows = 1u << (a.b1 + a.b2);
  const uint32_t per = (windows + kScanThreads - 1) / kScanThreads;
  const uint32_t first = threadIdx.x * per;
  const uint32_t* __restrict__ cnt = a.cnt_b;
  uint32_t* __restrict__ base = a.base_b;
  uint32_t total;
  if (per >= 4) {
    const u32x4* __restrict__ c4 = reinterpret_cast<const u32x4*>(cnt + first);
    u32x4* __restrict__ b4 = reinterpret_cast<u32x4*>(base + first);
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per / 4; ++i) {
      const u32x4 c = c4[i];
      sum += c.x + c.y + c.z + c.w;
    }
    uint32_t run = block_exclusive_scan<kScanThreads>(sum, waves, &total);
    for (uint32_t i = 0; i < per / 4; ++i) {
      const u32x4 c = c4[i];
      u32x4 b;
      b.x = run;
      b.y = run + c.x;
      b.z = b.y + c.y;
      b.w = b.z + c.z;
      run = b.w + c.w;
      b4[i] = b;
    }
  } else {
    // per is 1 or 2; with fewer windows than threads the rest own none
    const uint32_t mine = first < windows ? per : 0u;
    uint32_t c[2] = {0u, 0u};
    for (uint32_t i = 0; i < mine; ++i) c[i] = cnt[first + i];
    uint32_t run = block_exclusive_scan<kScanThreads>(c[0] + c[1], waves, &total);
    for (uint32_t i = 0; i < mine; ++i) {
      base[first + i] = run;
      run += c[i];
    }
  }
}

// Window bits per record size: the window's records fill 64 KB of LDS.
template <int EB>
constexpr uint32_t kWindowBits = EB == 1 ? 16 : EB == 2 ? 15 : EB == 4 ? 14 : EB == 8 ? 13 : 12;

// One workgroup per window q of 2^s padded indices at a time (persistent:
// windows gridDim.x apart): its records go to LDS at i mod 2^s with a kept
// bit; each thread owns 2^S / kPlaceThreads consecutive slots, counts its
// kept bits, takes its start from a workgroup scan, and moves its records to
// their ranks; the window is then written in order at out[base_b[q]].  The
// first kPrefetch entries per thread of the next window are loaded while the
// current one is ranked and written.  (s < S only when the whole domain is
// one window.)
constexpr uint32_t kPrefetch = 4;

// kPrefetch entries per thread of a window, from entry e0 on: entry
// e0 + j * T + tid (T threads), raw 16-bit slot and record.  The loads are
// unconditional (no branch per load: a load under a lane mask leaves its
// register pending for the compiler's wait counting, which then waits for
// it, and everything older, at the register's next write).  The slot is masked where it is used, not here: an
// operation on a loaded value right after its load would make the wavefront
// wait for the load at that point.  The pointers are plain (not restrict):
// loads through restrict pointers to data nothing writes may be moved past
// the workgroup barriers, which would undo the prefetch.
template <typename T>
__device__ __forceinline__ void load_window_batch(uint32_t (&il)[kPrefetch], T (&v)[kPrefetch], const uint16_t* wi,
                                                  const T* wv, uint32_t e0, uint32_t cnt) {
#pragma unroll
  for (uint32_t j = 0; j < kPrefetch; ++j) {
    const uint32_t e = e0 + j * kPlaceThreads + threadIdx.x;
    const uint32_t ec = e < cnt ? e : 0u;  // lanes past the count re-read entry 0 (inside the window)
    il[j] = wi[ec];
    v[j] = wv[ec];
  }
}

template <int EB>
__global__ __launch_bounds__(kPlaceThreads, 8) void staged_place_kernel(const StagedArgs a) {
  // records move as plain words here (16-byte records as one 4-word vector)
  using T = std::conditional_t<EB == 16, u32x4, typename Payload<EB>::T>;
  constexpr uint32_t S = kWindowBits<EB>;
  constexpr uint32_t W = 1u << S;
  constexpr uint32_t kPer = W / kPlaceThreads;  // slots per thread: 4 .. 64
  static_assert(kPer >= 4 && kPer <= 64, "slots per thread");
  __shared__ T vals[W];
  __shared__ uint32_t bits[W / 32];
  __shared__ uint32_t waves[kPlaceThreads / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t windows = 1u << (a.b1 + a.b2);
  // counts and bases are only read here: scalar loads, outside the vector
  // memory counter that the record loads and output stores share
  const ConstKeys cnts = global_keys(a.cnt_b);
  const ConstKeys bases = global_keys(a.base_b);
  uint32_t q = blockIdx.x;
  if (q >= windows) return;
  const uint16_t* wi = a.idx_b + (uint64_t(q) << a.s);
  const T* wv = reinterpret_cast<const T*>(a.val_b) + (uint64_t(q) << a.s);
  uint32_t il[kPrefetch];
  T hv[kPrefetch];
  uint32_t cnt = cnts[q];
  uint32_t next_cnt = q + gridDim.x < windows ? cnts[q + gridDim.x] : 0u;
  load_window_batch<T>(il, hv, wi, wv, 0, cnt);
  wait_vector_memory();  // both paths into the loop arrive with the head loaded
  for (;;) {
    const uint32_t base = bases[q];
    for (uint32_t t = tid; t < W / 32; t += kPlaceThreads) bits[t] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kPrefetch; ++j) {
      if (tid + j * kPlaceThreads < cnt) {
        const uint32_t x = il[j] & (W - 1);
        vals[x] = hv[j];
        atomicOr(&bits[x >> 5], 1u << (x & 31));
      }
    }
    // the rest of the window, kPrefetch entries per thread per batch, each
    // batch's loads issued together
    for (uint32_t e0 = kPrefetch * kPlaceThreads; e0 < cnt; e0 += kPrefetch * kPlaceThreads) {
      load_window_batch<T>(il, hv, wi, wv, e0, cnt);
#pragma unroll
      for (uint32_t j = 0; j < kPrefetch; ++j) {
        if (e0 + j * kPlaceThreads + tid < cnt) {
          const uint32_t x = il[j] & (W - 1);
          vals[x] = hv[j];
          atomicOr(&bits[x >> 5], 1u << (x & 31));
        }
      }
    }
    const uint32_t cur_cnt = cnt;
    const uint32_t next = q + gridDim.x;
    const bool more = next < windows;
    if (more) {
      // the next window's head goes out now and lands during the ranking
      cnt = next_cnt;
      next_cnt = next + gridDim.x < windows ? cnts[next + gridDim.x] : 0u;
      wi = a.idx_b + (uint64_t(next) << a.s);
      wv = reinterpret_cast<const T*>(a.val_b) + (uint64_t(next) << a.s);
      load_window_batch<T>(il, hv, wi, wv, 0, cnt);
      // keeps the compiler from sinking these loads to their use in the
      // next iteration (after the output stores)
      asm volatile("" ::: "memory");
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
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
      const uint64_t below = mine & ((uint64_t(1) << j) - 1u);
      if ((mine >> j) & 1u) vals[start + uint32_t(__builtin_popcountll(below))] = r[j];
    }
    __syncthreads();
    // the next window's head loads are in before the output stores go out
    wait_vector_memory();
    T* __restrict__ wo = reinterpret_cast<T*>(a.out) + base;
    for (uint32_t t = tid; t < cur_cnt; t += kPlaceThreads) wo[t] = vals[t];
    __syncthreads();
    if (!more) break;
    q = next;
  }
}

// The staged un-shuffle (the inverse of the shuffle, out[f(i)] = in[rank(i)]
// for every kept padded index i): the same distribution passes, keyed by the
// output position f(i) instead of the padded index.  Output positions are
// dense in [0, n), so the place pass's ranks are the positions themselves.
// First, per tile of TK padded indices: the forward cipher, the kept images
// compacted in index order at keys[tile * TK + e] and the tile's count.
template <int EB>
constexpr uint32_t kKeyTile = DistShape<EB, 3>::kTile;
// key tiles per distribution tile of the first pass's large shape (1 or 2)
template <int EB>
constexpr uint32_t kKeysPerTile = DistShape<EB, 1>::kTile / kKeyTile<EB>;

template <int EB, bool ODD>
__global__ __launch_bounds__(512) void staged_unshuffle_keys_kernel(const StagedArgs a, uint32_t* __restrict__ keys,
                                                                    uint32_t* __restrict__ tile_cnt) {
  constexpr uint32_t TK = kKeyTile<EB>;
  constexpr uint32_t kWaves = 8, kItems = TK / 512u;
  __shared__ uint32_t wave_total[kWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint64_t domain = uint64_t(1) << a.k;
  const uint64_t t = blockIdx.x;
  // wave w holds indices [w * 64 * kItems, (w + 1) * 64 * kItems) of the
  // tile, item j the 64 consecutive ones from j * 64: index order is (wave,
  // item, lane)
  const uint64_t first = t * TK + uint64_t(wave) * (64u * kItems) + lane;
  const uint32_t wmask24 = a.cs.wmask & 0xFFFFFFu;
  uint32_t L[kItems], R[kItems];
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    const uint64_t x = first + 64u * j;
    L[j] = uint32_t(x >> a.cs.r) & wmask24;
    R[j] = uint32_t(x);
  }
  vp_encrypt<ODD, kItems>(L, R, a.cs, a.rounds, a.key);
  uint32_t y[kItems], at[kItems], keep_bits = 0, run = 0;
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    y[j] = (L[j] << a.cs.r) | (R[j] & a.cs.rmask);
    const bool keep = first + 64u * j < domain && uint64_t(y[j]) < a.n;
    const uint64_t m = __ballot(keep);
    at[j] = run + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    run += uint32_t(__builtin_popcountll(m));
    keep_bits |= keep ? (1u << j) : 0u;
  }
  if (lane == 0) wave_total[wave] = run;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < kWaves; ++w) {
    const uint32_t c = wave_total[w];
    before += w < wave ? c : 0u;
    total += c;
  }
  uint32_t* __restrict__ kt = keys + t * TK;
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j)
    if ((keep_bits >> j) & 1u) kt[before + at[j]] = y[j];
  if (tid == 0) tile_cnt[t] = total;
}

// Then per kKeysPerTile consecutive key tiles (one workgroup each, the first
// pass's large tile shape): their kept images with the records
// in[tile_base[t] + e] (the tiles' ranks are consecutive, so the reads are
// too), distributed by the image's first digit like the first pass.
template <int EB>
__global__ __launch_bounds__((DistShape<EB, 1>::kThreads)) void staged_unshuffle_first_kernel(
    const StagedArgs a, const uint32_t* __restrict__ keys, const uint32_t* __restrict__ tile_cnt,
    const uint32_t* __restrict__ tile_base, uint32_t tiles) {
  using S = DistShape<EB, 1>;
  using T = typename Payload<EB>::T;
  constexpr uint32_t kItems = S::kItems;
  constexpr uint32_t TK = kKeyTile<EB>;
  __shared__ DistLds<EB, S> lds;
  const uint32_t tid = threadIdx.x;
  const uint64_t t = uint64_t(blockIdx.x) * kKeysPerTile<EB>;
  const uint32_t c0 = global_keys(tile_cnt)[t];
  const uint32_t c1 = kKeysPerTile<EB> == 2 && t + 1 < tiles ? global_keys(tile_cnt)[t + 1] : 0u;
  const uint32_t cnt = c0 + c1;
  if (cnt == 0) return;  // uniform across the workgroup
  const uint32_t base = global_keys(tile_base)[t];
  const uint32_t digits = 1u << a.b1;
  const uint32_t shift = a.k - a.b1;
  const uint64_t cap = uint64_t(1) << shift;
  const bool windows = a.b2 == 0;
  void* idx_out = windows ? static_cast<void*>(a.idx_b) : static_cast<void*>(a.idx_a);
  uint8_t* val_out = windows ? a.val_b : a.val_a;
  uint32_t* counts = windows ? a.cnt_b : a.cnt_a;
  for (uint32_t d = tid; d < digits; d += S::kThreads) lds.hist[d] = 0;
  T v[kItems];
  uint32_t ii[kItems], pos[kItems];
  uint32_t valid = 0;
  // entry e: key tile t's e-th image, then tile t + 1's (e - c0)-th
  const uint32_t* __restrict__ kt = keys + t * TK;
  const uint8_t* src = a.in + uint64_t(base) * EB;
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j) {
    const uint32_t off = j * S::kThreads + tid;
    const bool ok = off < cnt;
    valid |= ok ? (1u << j) : 0u;
    const uint32_t oc = ok ? off : 0u;  // idle lanes re-read the tile's first entry
    ii[j] = kt[oc < c0 ? oc : TK + (oc - c0)];
    v[j] = load_record<EB>(src + oc * uint32_t(EB), 0);
  }
  __syncthreads();  // the histogram is cleared
#pragma unroll
  for (uint32_t j = 0; j < kItems; ++j)
    pos[j] = ((valid >> j) & 1u) ? atomicAdd(&lds.hist[ii[j] >> shift], 1u) : 0u;
  __syncthreads();
  Reservation<S> res;
  reserve_runs<EB, S>(lds, res, digits, 0, counts);
  stage_entries<EB, S>(lds, ii, v, pos, valid, shift, digits);
  publish_bases<EB, S>(lds, res, digits, 0u, uint32_t(cap));
  if (windows)
    write_runs<EB, S, true>(lds, res.count, shift, digits, idx_out, val_out);
  else
    write_runs<EB, S, false>(lds, res.count, shift, digits, idx_out, val_out);
}

// Workgroups of fn that stay resident on the device at once.
uint32_t resident_groups(const void* fn, uint32_t threads, uint32_t num_cus) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, int(threads), 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return uint32_t(per_cu) * (num_cus ? num_cus : 1);
}

// First pass: persistent, as many workgroups as stay resident.
template <int EB, bool ODD, bool SMALL>
void launch_first(const StagedArgs& a, uint32_t num_cus, hipStream_t stream) {
  using S1 = DistShape<EB, SMALL ? 3 : 1>;
  const uint64_t tiles = (a.n + S1::kTile - 1) / S1::kTile;
  const uint64_t r1 =
      resident_groups(reinterpret_cast<const void*>(&staged_first_kernel<EB, ODD, SMALL>), S1::kThreads, num_cus);
  const dim3 g1(uint32_t(tiles < r1 ? tiles : r1));
  hipLaunchKernelGGL((staged_first_kernel<EB, ODD, SMALL>), g1, dim3(S1::kThreads), 0, stream, a);
}

template <int EB>
hipError_t launch_staged_rest(const StagedArgs& a, uint32_t num_cus, hipStream_t stream);

template <int EB>
hipError_t launch_staged_eb(const StagedArgs& a, bool odd, uint32_t num_cus, hipStream_t stream) {
  const uint32_t zero_groups = std::max(1u, std::min(256u, (1u << (a.b1 + a.b2)) / 256u));
  hipLaunchKernelGGL(staged_zero_kernel, dim3(zero_groups), dim3(256), 0, stream, a);
  // the two-workgroups-per-CU first pass once the inverse cipher is long
  // enough for overlap to pay (about 80 instructions: five per even-k round,
  // eight per odd-k round) and 2^b1 <= 256 keeps its runs long
  const bool small_ok = a.b1 <= 8 && a.rounds * (odd ? 8u : 5u) >= 80u;
  if (!odd) {
    if constexpr (EB <= 4) {
      if (small_ok)
        launch_first<EB, false, true>(a, num_cus, stream);
      else
        launch_first<EB, false, false>(a, num_cus, stream);
    } else {
      launch_first<EB, false, false>(a, num_cus, stream);
    }
  } else if constexpr (EB <= 4) {
    if (small_ok)
      launch_first<EB, true, true>(a, num_cus, stream);
    else
      launch_first<EB, true, false>(a, num_cus, stream);
  } else {
    launch_first<EB, true, false>(a, num_cus, stream);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_staged_rest<EB>(a, num_cus, stream);
}

// The passes after the first: second distribution, window scan, place.
template <int EB>
hipError_t launch_staged_rest(const StagedArgs& a, uint32_t num_cus, hipStream_t stream) {
  using S2 = DistShape<EB, 2>;
  hipError_t e;
  if (a.b2) {
    // second pass: one workgroup per work item (most of the empty ones exit at once)
    const uint64_t work = (uint64_t(1) << a.b1) * ((uint64_t(1) << (a.k - a.b1)) / S2::kTile);
    const dim3 g2{uint32_t(work)};
    hipLaunchKernelGGL((staged_second_kernel<EB>), g2, dim3(S2::kThreads), 0, stream, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(staged_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t windows = 1u << (a.b1 + a.b2);
  const uint32_t r3 = resident_groups(reinterpret_cast<const void*>(&staged_place_kernel<EB>), kPlaceThreads,
                                      num_cus);
  hipLaunchKernelGGL((staged_place_kernel<EB>), dim3(windows < r3 ? windows : r3), dim3(kPlaceThreads), 0, stream,
                     a);
  return hipGetLastError();
}

template <int EB>
hipError_t launch_unshuffle_eb(const StagedArgs& a, bool odd, uint32_t* keys, uint32_t* tile_cnt,
                               uint32_t* tile_base, uint32_t num_cus, hipStream_t stream) {
  using S = DistShape<EB, 1>;
  const uint64_t domain = uint64_t(1) << a.k;
  const uint32_t tiles = uint32_t(domain > kKeyTile<EB> ? domain / kKeyTile<EB> : 1u);  // a power of two
  const uint32_t zero_groups = std::max(1u, std::min(256u, (1u << (a.b1 + a.b2)) / 256u));
  hipLaunchKernelGGL(staged_zero_kernel, dim3(zero_groups), dim3(256), 0, stream, a);
  if (odd)
    hipLaunchKernelGGL((staged_unshuffle_keys_kernel<EB, true>), dim3(tiles), dim3(512), 0, stream, a, keys,
                       tile_cnt);
  else
    hipLaunchKernelGGL((staged_unshuffle_keys_kernel<EB, false>), dim3(tiles), dim3(512), 0, stream, a, keys,
                       tile_cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the tiles' first ranks: the window scan over the tile counts
  StagedArgs sc = a;
  sc.cnt_b = tile_cnt;
  sc.base_b = tile_base;
  sc.b1 = uint32_t(__builtin_ctz(tiles));
  sc.b2 = 0;
  hipLaunchKernelGGL(staged_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, sc);
  const uint32_t groups = (tiles + kKeysPerTile<EB> - 1) / kKeysPerTile<EB>;
  hipLaunchKernelGGL((staged_unshuffle_first_kernel<EB>), dim3(groups), dim3(S::kThreads), 0, stream, a, keys,
                     tile_cnt, tile_base, tiles);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_staged_rest<EB>(a, num_cus, stream);
}

}  // namespace

uint32_t unshuffle_key_tile(uint32_t elem_bytes) {
  switch (elem_bytes) {
    case 1: return kKeyTile<1>;
    case 2: return kKeyTile<2>;
    case 4: return kKeyTile<4>;
    case 8: return kKeyTile<8>;
    case 16: return kKeyTile<16>;
    default: return 0;
  }
}

hipError_t launch_unshuffle_staged(const StagedArgs& a, uint32_t* keys, uint32_t* tile_cnt, uint32_t* tile_base,
                                   uint32_t elem_bytes, uint32_t num_cus, hipStream_t stream) {
  const bool odd = ((a.cs.w + a.cs.r) & 1u) != 0;
  switch (elem_bytes) {
    case 1: return launch_unshuffle_eb<1>(a, odd, keys, tile_cnt, tile_base, num_cus, stream);
    case 2: return launch_unshuffle_eb<2>(a, odd, keys, tile_cnt, tile_base, num_cus, stream);
    case 4: return launch_unshuffle_eb<4>(a, odd, keys, tile_cnt, tile_base, num_cus, stream);
    case 8: return launch_unshuffle_eb<8>(a, odd, keys, tile_cnt, tile_base, num_cus, stream);
    case 16: return launch_unshuffle_eb<16>(a, odd, keys, tile_cnt, tile_base, num_cus, stream);
    default: return hipErrorInvalidValue;
  }
}

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
    *b1 = nb / 2 + 1 < kMaxDigitBits ? nb / 2 + 1 : kMaxDigitBits;
    *b2 = nb - *b1;
  }
  // the second pass reads first-pass buckets in whole distribution tiles
  if (*b2 && (uint64_t(1) << (k - *b1)) < kMaxFirstTile) return false;
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
